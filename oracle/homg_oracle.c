/*
 * homg_oracle.c -- plain FP64 CPU oracle for the high occupancy multigrid
 * (HOMG) of Becerra-Sagredo, Malaga and Mandujano, "A novel and scalable
 * multigrid algorithm for many-core architectures" (arXiv:1108.2045).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * path.  Everything is IEEE double, one node at a time, in the order the
 * paper states the operations; the OpenMP pragmas only split independent
 * node loops between threads and never change a result (the norm sums run
 * serially, in index order).
 *
 * Grids (Sec. 2, nested discretisations): d in {2,3}, n = 2^k + 1 nodes per
 * side on the unit square/cube, h = 1/(n-1).  Arrays are C-ordered with x
 * fastest: 2D node (j,i) at j*n + i, 3D node (k,j,i) at (k*n + j)*n + i.
 * Level m has stride l = 2^m and spacing h_l = l*h (Sec. 2, the level-m
 * relaxation); its lattice is the set of nodes whose every index is a
 * multiple of l.  Compact level-m arrays hold only the lattice: side
 * (n-1)/l + 1, same ordering.
 *
 * Operator (Sec. 2, the system A u = f): A = -div(a grad) discretised with
 * the 2d-point stencil; the face coefficient between nodes p and q is the
 * harmonic mean 2 a_p a_q / (a_p + a_q) of the nodal coefficient a, and
 * a == NULL means a = 1 everywhere (the plain -Laplacian, 5- or 7-point).
 * The paper writes the Poisson problem with the opposite sign (Sec. 4,
 * eq. "poisson"); the oracle uses the symmetric positive definite -Laplacian
 * and the Jacobi update with the sign that makes it converge (see the
 * relaxation below).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

static size_t node(int n, int k, int j, int i)
{
    return ((size_t)k * (size_t)n + (size_t)j) * (size_t)n + (size_t)i;
}

static int nz_of(int d, int n) { return d == 3 ? n : 1; }

/* A node is on the Dirichlet boundary if any of its d coordinates is 0 or
 * n-1.  In 2D the k index is always 0 and is not a coordinate. */
static int on_boundary(int d, int n, int k, int j, int i)
{
    if (i == 0 || i == n - 1 || j == 0 || j == n - 1) return 1;
    if (d == 3 && (k == 0 || k == n - 1)) return 1;
    return 0;
}

/* Face coefficient between nodes p and q: harmonic mean of the nodal
 * coefficient, 1 for the constant-coefficient Laplacian. */
static double face(const double *a, size_t p, size_t q)
{
    if (a == NULL) return 1.0;
    return 2.0 * a[p] * a[q] / (a[p] + a[q]);
}

/* The 2d neighbour offsets at distance l, in the fixed order
 * -x, +x, -y, +y, -z, +z. */
static void neighbours(int d, int l, int off[6][3])
{
    int t = 0;
    for (int axis = 0; axis < d; ++axis) {
        for (int s = -1; s <= 1; s += 2) {
            off[t][0] = off[t][1] = off[t][2] = 0;
            off[t][2 - axis] = s * l; /* [0]=k(z) [1]=j(y) [2]=i(x) */
            ++t;
        }
    }
}

/*
 * Residual r = f - A u (Sec. 2, two-level scheme step (b); Sec. 2 last
 * paragraph, the residual equation that restarts the cycles).  Interior nodes
 * only; r = 0 on the boundary.  Returns sum of r^2 over interior nodes,
 * accumulated in index order.
 */
double oracle_residual(int d, int n, const double *a, const double *f,
                       const double *u, double *r)
{
    const double h = 1.0 / (double)(n - 1);
    const double inv_h2 = 1.0 / (h * h);
    int off[6][3];
    neighbours(d, 1, off);
    const int nz = nz_of(d, n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t p = node(n, k, j, i);
                if (on_boundary(d, n, k, j, i)) { r[p] = 0.0; continue; }
                double au = 0.0;
                for (int t = 0; t < 2 * d; ++t) {
                    size_t q = node(n, k + off[t][0], j + off[t][1], i + off[t][2]);
                    au += face(a, p, q) * (u[p] - u[q]);
                }
                r[p] = f[p] - au * inv_h2;
            }
    double s = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                if (!on_boundary(d, n, k, j, i)) {
                    double v = r[node(n, k, j, i)];
                    s += v * v;
                }
    return s;
}

/* Sum of squares of f over interior nodes, in index order. */
double oracle_norm2_interior(int d, int n, const double *f)
{
    double s = 0.0;
    const int nz = nz_of(d, n);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                if (!on_boundary(d, n, k, j, i)) {
                    double v = f[node(n, k, j, i)];
                    s += v * v;
                }
    return s;
}

/*
 * One restriction step P (Sec. 2: restrictions are linearly weighted
 * averages of neighbouring sources, organised as nested partial reductions).
 * Full weighting: coarse node I takes sum over o in {-1,0,1}^d of
 * prod_axis w(o_axis) * rf[2I + o], with w(0) = 1/2 and w(+-1) = 1/4.
 * Coarse boundary nodes are 0.  nf is the fine side; the coarse side is
 * (nf-1)/2 + 1.  P_m (the level-m restriction of the paper) is this step
 * applied m times.
 */
void oracle_restrict(int d, int nf, const double *rf, double *rc)
{
    const int nc = (nf - 1) / 2 + 1;
    const int nzc = nz_of(d, nc);
#pragma omp parallel for schedule(static)
    for (int K = 0; K < nzc; ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < nc; ++I) {
                size_t P = node(nc, K, J, I);
                if (on_boundary(d, nc, K, J, I)) { rc[P] = 0.0; continue; }
                double s = 0.0;
                int zlo = (d == 3) ? -1 : 0, zhi = (d == 3) ? 1 : 0;
                for (int oz = zlo; oz <= zhi; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            double w = (ox == 0 ? 0.5 : 0.25) * (oy == 0 ? 0.5 : 0.25);
                            if (d == 3) w *= (oz == 0 ? 0.5 : 0.25);
                            int kf = (d == 3) ? 2 * K + oz : 0;
                            s += w * rf[node(nf, kf, 2 * J + oy, 2 * I + ox)];
                        }
                rc[P] = s;
            }
}

/*
 * Interpolation S from the level-m lattice (Sec. 2: interpolations are
 * linear).  The value at node (k,j,i) is the multilinear interpolant of the
 * 2^d lattice values at the corners of the level-m cell that contains it:
 * corner c = floor(index / l) * l per axis, weight t = (index - c) / l, and
 * the far corner c + l.  Lattice nodes reproduce their own value.
 */
double oracle_interpolate(int d, int n, int m, const double *e, int k, int j, int i)
{
    const int l = 1 << m;
    const int ci = (i / l) * l, cj = (j / l) * l, ck = (d == 3) ? (k / l) * l : 0;
    const double ti = (double)(i - ci) / (double)l;
    const double tj = (double)(j - cj) / (double)l;
    const double tk = (d == 3) ? (double)(k - ck) / (double)l : 0.0;
    double v = 0.0;
    const int bz_hi = (d == 3) ? 1 : 0;
    for (int bz = 0; bz <= bz_hi; ++bz)
        for (int by = 0; by <= 1; ++by)
            for (int bx = 0; bx <= 1; ++bx) {
                double w = (bx ? ti : 1.0 - ti) * (by ? tj : 1.0 - tj);
                if (d == 3) w *= (bz ? tk : 1.0 - tk);
                if (w == 0.0) continue; /* the far corner of a cell edge may lie past the grid */
                v += w * e[node(n, ck + bz * l, cj + by * l, ci + bx * l)];
            }
    return v;
}

/*
 * Damped Jacobi relaxation at an interior level-m lattice node (Sec. 2, the
 * explicit Euler step of du/dt = kappa (L(u) - f) with stride l = 2^m and
 * spacing h_l = 2^m h).  For A e = r_m:
 *     e' = e + omega * (h_l^2 r_m - sum_q a_pq (e_p - e_q)) / sum_q a_pq
 * over the 2d lattice neighbours q = p +- l.  With a = 1 this is
 *     e' = e + (omega / 2d) (h_l^2 r_m - (2d e_p - sum_q e_q)),
 * the paper's update with the bracket's sign taken so that the fixed point
 * is the solution of the level-m system (the printed sign is reversed).
 * rm is the compact level-m residual, so its node is (k/l, j/l, i/l).
 */
static double relax_node(int d, int n, int m, double omega, const double *a,
                         const double *rm, const double *e, int k, int j, int i)
{
    const int l = 1 << m;
    const int nm = (n - 1) / l + 1;
    const double hl = (double)l / (double)(n - 1);
    int off[6][3];
    neighbours(d, l, off);
    size_t p = node(n, k, j, i);
    double sum_a = 0.0, flux = 0.0;
    for (int t = 0; t < 2 * d; ++t) {
        size_t q = node(n, k + off[t][0], j + off[t][1], i + off[t][2]);
        double apq = face(a, p, q);
        sum_a += apq;
        flux += apq * (e[p] - e[q]);
    }
    double rv = rm[node(nm, (d == 3) ? k / l : 0, j / l, i / l)];
    return e[p] + omega * (hl * hl * rv - flux) / sum_a;
}

/*
 * One HOMG iteration at level m over the whole grid (Sec. 2: relaxations and
 * interpolations fused into one task acting on complementary subsets of one
 * array; the HOMG steps (a)-(c)).  Every node reads only the previous iterate
 * e_old, so the interpolated nodes see the lattice values of the iteration
 * before (Sec. 4, Fig. 3 discussion: the interpolations are delayed one
 * iteration).  For every node p:
 *     boundary                 -> 0
 *     interior lattice node    -> relaxation (relax_node)
 *     any other node           -> S_m(e_old)(p)
 */
void oracle_sweep(int d, int n, int m, double omega, const double *a,
                  const double *rm, const double *e_old, double *e_new)
{
    const int l = 1 << m;
    const int nz = nz_of(d, n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t p = node(n, k, j, i);
                if (on_boundary(d, n, k, j, i)) { e_new[p] = 0.0; continue; }
                int lattice = (i % l == 0) && (j % l == 0) && (d == 2 || k % l == 0);
                if (lattice)
                    e_new[p] = relax_node(d, n, m, omega, a, rm, e_old, k, j, i);
                else
                    e_new[p] = oracle_interpolate(d, n, m, e_old, k, j, i);
            }
}

/* v <- v + e on every node (Sec. 2, two-level scheme step (d), and the
 * residual-equation restart of the last paragraph of Sec. 2). */
void oracle_add(int d, int n, double *v, const double *e)
{
    size_t total = (size_t)nz_of(d, n) * (size_t)n * (size_t)n;
    for (size_t p = 0; p < total; ++p) v[p] += e[p];
}

/* S_m applied at every node: out(p) = multilinear interpolant of the level-m
 * lattice values of e (lattice nodes reproduce their own value). */
void oracle_prolong(int d, int n, int m, const double *e, double *out)
{
    const int nz = nz_of(d, n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                out[node(n, k, j, i)] = oracle_interpolate(d, n, m, e, k, j, i);
}
