/*
 * pow2_oracle.c -- plain FP64 CPU oracle of the power-of-two grid strategy
 * of HOMG (Becerra-Sagredo, Malaga and Mandujano, arXiv:1108.2045, Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY (like homg_oracle.c): the product library never
 * calls, links or loads it.  Plain IEEE double, one node at a time.
 *
 * Grid: 2D, N = 2^k nodes per side (k >= 2) on the unit square, node (j,i)
 * at (i h, j h), h = 1/(N-1); nodes with i or j in {0, N-1} carry the zero
 * Dirichlet data.  The fine operator is the 5-point -Laplacian (the residual
 * of homg_oracle.c serves any side).  Sec. 3 leaves the details to a
 * missing figure; the reading implemented here:
 *
 *  - Four subdomains (quadrants) of N/2 nodes per side.  Quadrant (sx, sy)
 *    owns the nodes with (i >= N/2) == sx and (j >= N/2) == sy; its external
 *    corner is at index 0 (side 0) or N-1 (side 1) of each axis, and the
 *    local coordinate of index x on side s is a = x (s = 0) or N-1-x (s = 1).
 *  - Level m >= 1 (stride l = 2^m, spacing h_l = l h): quadrant (sx, sy)
 *    marks the nodes whose local coordinates are both multiples of l in
 *    [0, N/2] -- measured from its external corner, and up to N/2, one index
 *    past its own N/2 nodes: the points just outside the subdomain.  Without
 *    them the coarsest level (l = N/2) would have no interior point.  On
 *    every axis a marked index of side 0 is even and one of side 1 is odd,
 *    so the four sets are disjoint.
 *  - An iteration at level m >= 1 (the fused task of Sec. 2): every
 *    interior marked node relaxes (damped Jacobi with the 5-point stencil at
 *    distance l on the whole grid; a neighbour index outside [0, N-1] reads
 *    0), with its quadrant's restricted residual; every other interior node
 *    takes the bilinear interpolant, from the previous iterate, of the four
 *    marks of its own quadrant at the corners of the level-m cell holding it
 *    (no interpolation across subdomains).  Level 0 is damped Jacobi at
 *    every interior node.
 *  - Restriction: each quadrant has its own nested sequence, anchored at its
 *    external corner.  Family (sx, sy) at level 0 is r_0 seen from that
 *    corner (F_0[b][a] = r_0 at the global indices of local (a, b)); level j
 *    is the full weighting of level j-1 (weights 1/4, 1/2, 1/4 per axis at
 *    local 2A-1, 2A, 2A+1), side N / 2^j, with local index 0 -- the domain
 *    boundary -- held at 0.  Level j of a family covers the whole square (its
 *    last index N/2^j - 1 is interior), so the marks just outside the
 *    subdomain get a full stencil too.
 *
 * Arrays: whole-grid arrays are N x N, C order, x fastest.  Family arrays
 * of level j are s x s with s = N >> j, index [B * s + A] for local (A, B)
 * in units of 2^j.  Family index q = 2 sy + sx.
 */
#include <math.h>
#include <stddef.h>

static size_t at(int n, int j, int i) { return (size_t)j * (size_t)n + (size_t)i; }

/* Local coordinate of global index x on side s. */
static int local_of(int N, int s, int x) { return s ? N - 1 - x : x; }

/* Side (0 or 1) whose level-l mark set holds index x, or -1. */
static int mark_side(int N, int l, int x)
{
    for (int s = 0; s <= 1; ++s) {
        int a = local_of(N, s, x);
        if (a % l == 0 && a <= N / 2) return s;
    }
    return -1;
}

/* Family level 0: r0 seen from the corner of quadrant (sx, sy). */
void oracle_p2_family_base(int N, int sx, int sy, const double *r0, double *F)
{
    for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a)
            F[at(N, b, a)] = r0[at(N, local_of(N, sy, b), local_of(N, sx, a))];
}

/* One full-weighting step of a family: side nf -> nf / 2. */
void oracle_p2_restrict(int nf, const double *F, double *C)
{
    const int nc = nf / 2;
    for (int B = 0; B < nc; ++B)
        for (int A = 0; A < nc; ++A) {
            if (A == 0 || B == 0) { C[at(nc, B, A)] = 0.0; continue; }
            double s = 0.0;
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    double w = (ox == 0 ? 0.5 : 0.25) * (oy == 0 ? 0.5 : 0.25);
                    s += w * F[at(nf, 2 * B + oy, 2 * A + ox)];
                }
            C[at(nc, B, A)] = s;
        }
}

static double ev(int N, const double *e, int j, int i)
{
    if (i < 0 || j < 0 || i >= N || j >= N) return 0.0;
    return e[at(N, j, i)];
}

/* Bilinear interpolant at (j, i) from the level-l marks of the quadrant that
 * owns (j, i). */
static double interp(int N, int l, const double *e, int j, int i)
{
    const int sx = i >= N / 2, sy = j >= N / 2;
    const int ax = local_of(N, sx, i), ay = local_of(N, sy, j);
    const int cx = (ax / l) * l, cy = (ay / l) * l;
    const double tx = (double)(ax - cx) / (double)l, ty = (double)(ay - cy) / (double)l;
    double v = 0.0;
    for (int by = 0; by <= 1; ++by)
        for (int bx = 0; bx <= 1; ++bx) {
            double w = (bx ? tx : 1.0 - tx) * (by ? ty : 1.0 - ty);
            if (w == 0.0) continue;
            v += w * e[at(N, local_of(N, sy, cy + by * l), local_of(N, sx, cx + bx * l))];
        }
    return v;
}

/*
 * One whole-grid iteration at level m.  fam[q] is the level-m array of
 * family q (side N >> m); at m = 0, fam[0] is r0 itself (N x N, not
 * mirrored) and the others are unused.
 */
void oracle_p2_sweep(int N, int m, double omega, const double *const *fam,
                     const double *e_old, double *e_new)
{
    const int l = 1 << m;
    const double hl = (double)l / (double)(N - 1);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            size_t p = at(N, j, i);
            if (i == 0 || j == 0 || i == N - 1 || j == N - 1) { e_new[p] = 0.0; continue; }
            int sx = 0, sy = 0;
            double rv;
            if (m == 0) {
                rv = fam[0][p];
            } else {
                sx = mark_side(N, l, i);
                sy = mark_side(N, l, j);
                if (sx < 0 || sy < 0) { e_new[p] = interp(N, l, e_old, j, i); continue; }
                const int s = N >> m;
                rv = fam[2 * sy + sx][at(s, local_of(N, sy, j) / l, local_of(N, sx, i) / l)];
            }
            double c = e_old[p];
            double nb = ev(N, e_old, j, i - l) + ev(N, e_old, j, i + l) + ev(N, e_old, j - l, i) +
                        ev(N, e_old, j + l, i);
            e_new[p] = c + (omega / 4.0) * (hl * hl * rv - (4.0 * c - nb));
        }
}

/* The level-m mark map: 1 + q at a node marked by quadrant q, 0 elsewhere
 * (boundary nodes included). */
void oracle_p2_marks(int N, int m, int *out)
{
    const int l = 1 << m;
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            int sx = mark_side(N, l, i), sy = mark_side(N, l, j);
            out[at(N, j, i)] = (sx < 0 || sy < 0) ? 0 : 1 + 2 * sy + sx;
        }
}

/* The interpolation operator alone: every node takes the bilinear
 * interpolant from its own quadrant's level-m marks (marks reproduce their
 * own value). */
void oracle_p2_prolong(int N, int m, const double *e, double *out)
{
    const int l = 1 << m;
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i)
            out[at(N, j, i)] = interp(N, l, e, j, i);
}
