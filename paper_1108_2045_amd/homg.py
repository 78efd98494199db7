"""Thin ctypes binding of libhomg.so (the C ABI declared in include/homg.h).

Argument marshalling only: tensors are passed as device pointers, the
current torch stream as the hipStream_t, and every step of the method runs
in the library's HIP kernels.  There is no fallback: if the library is
missing or fails to load, importing this module raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhomg.so")

HOMG_OK = 0
STATUS_NAMES = {
    0: "HOMG_OK", 1: "HOMG_ERR_INVALID_ARG", 2: "HOMG_ERR_UNSUPPORTED", 3: "HOMG_ERR_OOM",
    4: "HOMG_ERR_WORKSPACE", 5: "HOMG_ERR_HIP", 6: "HOMG_ERR_NUMERICAL", 7: "HOMG_ERR_NOT_CONVERGED",
}
LAPLACE_5PT_2D, LAPLACE_7PT_3D, DIFFUSION_5PT_2D = 0, 1, 2
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
GRID_LAYOUTS = {"nested": 0, "pow2": 1}
RESTRICTIONS = {"pyramid": 0, "in_cycle": 1}


class HomgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("omega", ctypes.c_double),
                ("max_i", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("schedule", ctypes.POINTER(ctypes.c_int)), ("schedule_len", ctypes.c_int),
                ("precision", ctypes.c_int), ("temporal_block", ctypes.c_int),
                ("grid_layout", ctypes.c_int), ("restriction", ctypes.c_int), ("reserved", ctypes.c_int * 5)]


class Info(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("converged", ctypes.c_int),
                ("relres0", ctypes.c_double), ("final_relres", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int),
                ("sweeps", ctypes.c_longlong), ("launches", ctypes.c_longlong),
                ("host_syncs", ctypes.c_int), ("smoother_fell_back", ctypes.c_int)]


class TrainOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("steps", ctypes.c_int), ("batch", ctypes.c_int),
                ("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("seed", ctypes.c_uint64), ("reserved", ctypes.c_int * 8)]


SMOOTHER_WEIGHTS = 576
JACOBI, LEARNED = 0, 1


class KernelTime(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("level", ctypes.c_int), ("mode", ctypes.c_int),
                ("reserved", ctypes.c_int), ("launches", ctypes.c_longlong), ("ms", ctypes.c_double)]


KIND_NAMES = {0: "norm", 1: "residual", 2: "finalize", 3: "restrict", 4: "sweep",
              5: "gather", 6: "lattice", 7: "level_write", 8: "learned", 9: "transfer", 10: "tail"}


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libhomg.so not built (run __graft_entry__.build() or "
                          "python -m paper_1108_2045_amd.build): " + path)
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)
    H = ctypes.c_void_p
    L.homg_options_init.argtypes = [ctypes.POINTER(Options)]
    L.homg_options_init.restype = None
    L.homg_create.argtypes = [ctypes.POINTER(H), ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                              ctypes.c_int, ctypes.c_int, ctypes.POINTER(Options)]
    L.homg_destroy.argtypes = [H]
    L.homg_set_coefficient.argtypes = [H, dp, vp]
    L.homg_solve.argtypes = [H, dp, dp, ctypes.c_double, vp, ctypes.POINTER(Info)]
    L.homg_solve_cycles.argtypes = [H, dp, dp, ctypes.c_int, vp, ctypes.POINTER(Info)]
    L.homg_residual.argtypes = [H, dp, dp, dp, ctypes.POINTER(ctypes.c_double), vp]
    L.homg_get_schedule.argtypes = [H, ip, ctypes.c_int, ip]
    L.homg_step_restrict.argtypes = [H, ctypes.c_int, dp, dp, vp]
    L.homg_step_sweeps.argtypes = [H, ctypes.c_int, ctypes.c_int, dp, dp, dp, vp]
    L.homg_step_cycle.argtypes = [H, dp, dp, vp]
    L.homg_set_profiling.argtypes = [H, ctypes.c_int]
    L.homg_get_profile.argtypes = [H, ctypes.POINTER(KernelTime), ctypes.c_int, ip]
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.homg_batch_create.argtypes = [ctypes.POINTER(H), ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(Options)]
    L.homg_batch_solve.argtypes = [H, PP, PP, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_double),
                                   ip, ip]
    L.homg_batch_set_tile_rows.argtypes = [H, ctypes.c_int64, ctypes.c_int]
    L.homg_batch_set_pass_iters.argtypes = [H, ctypes.c_int64, ctypes.c_int]
    L.homg_batch_tune.argtypes = [H, PP, PP, ctypes.c_double, vp, ctypes.c_char_p]
    L.homg_batch_destroy.argtypes = [H]
    L.homg_set_smoother.argtypes = [H, ctypes.c_int, vp, ctypes.c_double, vp]
    L.homg_get_smoother_weights.argtypes = [H, vp, vp]
    L.homg_smoother_gate.argtypes = [H, ctypes.c_int, PP, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ip]
    L.homg_train_options_init.argtypes = [ctypes.POINTER(TrainOptions)]
    L.homg_train_options_init.restype = None
    L.homg_trainer_create.argtypes = [ctypes.POINTER(H)]
    L.homg_trainer_add_problem.argtypes = [H, H, dp, ctypes.c_int, vp]
    L.homg_trainer_count.argtypes = [H, ip]
    L.homg_trainer_train.argtypes = [H, vp, ctypes.POINTER(TrainOptions), vp,
                                     ctypes.POINTER(ctypes.c_double), vp]
    L.homg_trainer_loss.argtypes = [H, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.homg_trainer_destroy.argtypes = [H]
    L.homg_learn_forward.argtypes = [ctypes.c_int, ctypes.c_double, vp, vp, vp, vp, vp, vp]
    L.homg_learn_grad.argtypes = [ctypes.c_int, ctypes.c_double, vp, vp, vp, vp, vp, vp,
                                  ctypes.POINTER(ctypes.c_double), vp]
    L.homg_learn_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, vp, vp]
    L.homg_l1_error.argtypes = [H, dp, dp, ctypes.POINTER(ctypes.c_double), vp]
    L.homg_workspace_bytes.argtypes = [H, ctypes.POINTER(ctypes.c_size_t)]
    L.homg_trace_cycle.argtypes = [H, dp, dp, dp, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ip, vp]
    L.homg_residual_noalloc.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, dp,
                                        ctypes.POINTER(ctypes.c_double), vp]
    L.homg_last_error.argtypes = [H]
    L.homg_last_error.restype = ctypes.c_char_p
    L.homg_version.argtypes = []
    L.homg_version.restype = ctypes.c_char_p
    for name in ("homg_create", "homg_destroy", "homg_set_coefficient", "homg_solve",
                 "homg_solve_cycles", "homg_residual", "homg_get_schedule", "homg_step_restrict",
                 "homg_step_sweeps", "homg_step_cycle", "homg_set_profiling", "homg_get_profile",
                 "homg_batch_create", "homg_batch_solve", "homg_batch_set_tile_rows", "homg_batch_set_pass_iters",
                 "homg_batch_tune",
                 "homg_batch_destroy", "homg_set_smoother", "homg_get_smoother_weights",
                 "homg_smoother_gate", "homg_trainer_create", "homg_trainer_add_problem",
                 "homg_trainer_count", "homg_trainer_train", "homg_trainer_loss", "homg_trainer_destroy",
                 "homg_learn_forward", "homg_learn_grad", "homg_learn_adam", "homg_residual_noalloc",
                 "homg_l1_error", "homg_trace_cycle", "homg_workspace_bytes"):
        getattr(L, name).restype = ctypes.c_int
    return L


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _ptr(t, dtype=None):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("arrays must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("arrays must be contiguous (C order, x fastest)")
    want = dtype or torch.float64
    if t.dtype != want:
        raise ValueError("arrays must be %s" % str(want).replace("torch.", ""))
    return ctypes.c_void_p(t.data_ptr())


def _shape(t, shape, what):
    """Raise ValueError unless tensor t (if given) has exactly `shape`.  The C
    ABI takes raw pointers and cannot see sizes: an undersized array would
    be read or written past its end by the kernels."""
    if t is None:
        return
    if tuple(t.shape) != tuple(int(v) for v in shape):
        raise ValueError("%s must have shape %s, got %s" % (what, tuple(shape), tuple(t.shape)))


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One HOMG solver for a d-dimensional grid of side n = 2^k + 1."""

    def __init__(self, ndim, n, levels=0, stencil=None, omega=0.0, max_i=4, max_cycles=200,
                 schedule=None, precision="fp64", temporal_block=2, grid_layout="nested",
                 restriction="pyramid"):
        L = lib()
        if stencil is None:
            stencil = LAPLACE_5PT_2D if ndim == 2 else LAPLACE_7PT_3D
        opt = Options()
        L.homg_options_init(ctypes.byref(opt))
        opt.omega = omega
        opt.max_i = max_i
        opt.max_cycles = max_cycles
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt.temporal_block = temporal_block
        opt.grid_layout = GRID_LAYOUTS[grid_layout] if isinstance(grid_layout, str) else int(grid_layout)
        opt.restriction = RESTRICTIONS[restriction] if isinstance(restriction, str) else int(restriction)
        self._sched_buf = None
        if schedule is not None:
            flat = [int(v) for pair in schedule for v in pair]
            self._sched_buf = (ctypes.c_int * len(flat))(*flat)
            opt.schedule = self._sched_buf
            opt.schedule_len = len(schedule)
        dims = (ctypes.c_int64 * ndim)(*([n] * ndim))
        h = ctypes.c_void_p()
        st = L.homg_create(ctypes.byref(h), ndim, dims, levels, stencil, ctypes.byref(opt))
        if st != HOMG_OK:
            raise HomgError(st, L.homg_last_error(None).decode())
        self._h = h
        self.ndim, self.n, self.max_cycles = ndim, n, max_cycles
        self.precision = precision
        self.pow2 = opt.grid_layout == GRID_LAYOUTS["pow2"]

    def _check(self, st):
        if st != HOMG_OK:
            raise HomgError(st, lib().homg_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().homg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _grid(self, level=0):
        return ((self.n - 1) // (1 << level) + 1,) * self.ndim

    def _level(self, level):
        if getattr(self, "pow2", False):
            return  # the library refuses the nested-only step entry points
        side = (self.n - 1) // (1 << level) + 1 if level >= 0 else 0
        if level < 0 or side < 3 or (side - 1) << level != self.n - 1:
            raise ValueError("level %d out of range for side %d" % (level, self.n))

    def set_coefficient(self, a, stream=None):
        _shape(a, self._grid(), "a")
        self._check(lib().homg_set_coefficient(self._h, _ptr(a), _stream(stream)))

    def _info(self):
        info = Info()
        hist = (ctypes.c_double * (self.max_cycles + 1))()
        info.history = hist
        info.history_cap = self.max_cycles + 1
        return info, hist

    @staticmethod
    def _result(info, hist):
        return {"cycles": info.cycles, "converged": bool(info.converged), "relres0": info.relres0,
                "final_relres": info.final_relres, "history": list(hist[:info.cycles + 1]),
                "sweeps": info.sweeps, "launches": info.launches, "host_syncs": info.host_syncs,
                "smoother_fell_back": bool(info.smoother_fell_back)}

    def solve(self, f, u, tol=1e-10, stream=None, raise_on_status=True):
        _shape(f, self._grid(), "f")
        _shape(u, self._grid(), "u")
        info, hist = self._info()
        st = lib().homg_solve(self._h, _ptr(f), _ptr(u), tol, _stream(stream), ctypes.byref(info))
        out = self._result(info, hist)
        out["status"] = st
        if raise_on_status:
            self._check(st)
        return out

    def solve_cycles(self, f, u, cycles, stream=None):
        _shape(f, self._grid(), "f")
        _shape(u, self._grid(), "u")
        info, hist = self._info()
        st = lib().homg_solve_cycles(self._h, _ptr(f), _ptr(u), cycles, _stream(stream), ctypes.byref(info))
        self._check(st)
        return self._result(info, hist)

    def residual(self, f, u, r=None, stream=None):
        for t, what in ((f, "f"), (u, "u"), (r, "r")):
            _shape(t, self._grid(), what)
        rel = ctypes.c_double()
        self._check(lib().homg_residual(self._h, _ptr(f), _ptr(u), _ptr(r), ctypes.byref(rel), _stream(stream)))
        return rel.value

    def l1_error(self, u_ref, v, stream=None):
        """Normalised L1 error sum|u_ref - v| / sum|u_ref| (Sec. 4), computed on the GPU."""
        _shape(u_ref, self._grid(), "u_ref")
        _shape(v, self._grid(), "v")
        err = ctypes.c_double()
        self._check(lib().homg_l1_error(self._h, _ptr(u_ref), _ptr(v), ctypes.byref(err), _stream(stream)))
        return err.value

    def trace_cycle(self, f, u, u_ref, stream=None):
        """One MFMG cycle from e = 0, one whole-grid iteration at a time: the
        normalised L1 error of u + e after every iteration (one WU each); u
        receives u + e at the end."""
        for t, what in ((f, "f"), (u, "u"), (u_ref, "u_ref")):
            _shape(t, self._grid(), what)
        cap = sum(it for _, it in self.schedule())
        buf = (ctypes.c_double * max(cap, 1))()
        cnt = ctypes.c_int()
        self._check(lib().homg_trace_cycle(self._h, _ptr(f), _ptr(u), _ptr(u_ref), buf, cap, ctypes.byref(cnt),
                                           _stream(stream)))
        return list(buf[:cnt.value])

    def workspace_bytes(self):
        """Device memory held by the handle (not counting the caller's arrays)."""
        v = ctypes.c_size_t()
        self._check(lib().homg_workspace_bytes(self._h, ctypes.byref(v)))
        return v.value

    def schedule(self):
        n = ctypes.c_int()
        self._check(lib().homg_get_schedule(self._h, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_int * (2 * n.value))()
        self._check(lib().homg_get_schedule(self._h, buf, n.value, ctypes.byref(n)))
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(n.value)]

    def set_profiling(self, enable=True):
        self._check(lib().homg_set_profiling(self._h, 1 if enable else 0))

    def profile(self):
        """[{kind, level, mode, launches, ms}] accumulated since profiling was enabled."""
        n = ctypes.c_int()
        self._check(lib().homg_get_profile(self._h, None, 0, ctypes.byref(n)))
        buf = (KernelTime * max(n.value, 1))()
        self._check(lib().homg_get_profile(self._h, buf, n.value, ctypes.byref(n)))
        return [{"kind": KIND_NAMES.get(b.kind, b.kind), "level": b.level, "mode": b.mode,
                 "launches": b.launches, "ms": b.ms} for b in buf[:n.value]]

    def step_restrict(self, level, r_fine, r_coarse, stream=None):
        self._level(level)
        self._level(level + 1)
        if not getattr(self, "pow2", False):
            _shape(r_fine, self._grid(level), "r_fine")
            _shape(r_coarse, self._grid(level + 1), "r_coarse")
        self._check(lib().homg_step_restrict(self._h, level, _ptr(r_fine), _ptr(r_coarse), _stream(stream)))

    def step_sweeps(self, level, iters, e_old, r_level, e_new, stream=None):
        self._level(level)
        _shape(e_old, self._grid(), "e_old")
        if not getattr(self, "pow2", False):
            _shape(r_level, self._grid(level), "r_level")
        _shape(e_new, self._grid(), "e_new")
        self._check(lib().homg_step_sweeps(self._h, level, iters, _ptr(e_old), _ptr(r_level),
                                           _ptr(e_new), _stream(stream)))

    def step_cycle(self, r0, acc, stream=None):
        _shape(r0, self._grid(), "r0")
        _shape(acc, self._grid(), "acc")
        self._check(lib().homg_step_cycle(self._h, _ptr(r0), _ptr(acc), _stream(stream)))

    def set_smoother(self, smoother, w=None, fallback_ratio=0.0, stream=None):
        """smoother: JACOBI or LEARNED; w: 576 float32 weights on the GPU (rounded to BF16)."""
        import torch
        wp = _ptr(_weights(w), torch.float32) if w is not None else None
        self._check(lib().homg_set_smoother(self._h, int(smoother), wp, fallback_ratio, _stream(stream)))

    def smoother_weights(self, stream=None):
        """The FP32 values of the BF16 weights in use (a new GPU tensor)."""
        import torch
        out = torch.empty(SMOOTHER_WEIGHTS, dtype=torch.float32, device="cuda")
        self._check(lib().homg_get_smoother_weights(self._h, _ptr(out, torch.float32), _stream(stream)))
        return out

    def smoother_gate(self, fs, cycles, stream=None):
        for f in fs:
            _shape(f, self._grid(), "f")
        n = len(fs)
        arr = (ctypes.c_void_p * n)(*[_ptr(f).value for f in fs])
        rl = (ctypes.c_double * n)()
        rj = (ctypes.c_double * n)()
        acc = ctypes.c_int()
        self._check(lib().homg_smoother_gate(self._h, n, arr, cycles, _stream(stream), rl, rj, ctypes.byref(acc)))
        return {"accepted": bool(acc.value), "rho_learned": list(rl), "rho_jacobi": list(rj)}


def jacobi_weights(omega, device="cuda"):
    """A float32 weight vector whose network is exactly omega * rho (damped
    Jacobi): hidden channels 0 and 1 take +rho and -rho at the centre tap,
    and the output combines them with +omega and -omega."""
    import torch
    w = torch.zeros(SMOOTHER_WEIGHTS, dtype=torch.float32)
    w[0 * 27 + 0 * 9 + 4] = 1.0
    w[1 * 27 + 0 * 9 + 4] = -1.0
    w[432 + 0 * 9 + 4] = omega
    w[432 + 1 * 9 + 4] = -omega
    return w.to(device)


def _weights(w):
    if tuple(w.shape) != (SMOOTHER_WEIGHTS,):
        raise ValueError("the smoother has %d weights" % SMOOTHER_WEIGHTS)
    return w


class Trainer:
    """Training of the learned relaxation on pairs generated by plain HOMG."""

    def __init__(self):
        h = ctypes.c_void_p()
        st = lib().homg_trainer_create(ctypes.byref(h))
        if st != HOMG_OK:
            raise HomgError(st, lib().homg_last_error(None).decode())
        self._h = h

    def _check(self, st):
        if st != HOMG_OK:
            raise HomgError(st, lib().homg_last_error(None).decode())

    def add_problem(self, solver, f, cycles=1, stream=None):
        self._check(lib().homg_trainer_add_problem(self._h, solver._h, _ptr(f), cycles, _stream(stream)))

    def count(self):
        n = ctypes.c_int()
        self._check(lib().homg_trainer_count(self._h, ctypes.byref(n)))
        return n.value

    def train(self, w0, steps=300, batch=8, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0,
              stream=None):
        """Returns (FP32 values of the trained BF16 weights, per-step batch losses)."""
        import torch
        opt = TrainOptions()
        lib().homg_train_options_init(ctypes.byref(opt))
        opt.steps, opt.batch, opt.lr, opt.beta1, opt.beta2, opt.eps, opt.seed = (
            steps, batch, lr, beta1, beta2, eps, seed)
        out = torch.empty(SMOOTHER_WEIGHTS, dtype=torch.float32, device="cuda")
        hist = (ctypes.c_double * steps)()
        self._check(lib().homg_trainer_train(self._h, _ptr(_weights(w0), torch.float32), ctypes.byref(opt),
                                             _ptr(out, torch.float32), hist, _stream(stream)))
        return out, list(hist)

    def loss(self, w, stream=None):
        import torch
        v = ctypes.c_double()
        self._check(lib().homg_trainer_loss(self._h, _ptr(_weights(w), torch.float32), ctypes.byref(v),
                                            _stream(stream)))
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            lib().homg_trainer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_global(st):
    if st != HOMG_OK:
        raise HomgError(st, lib().homg_last_error(None).decode())


def _lattice(x, *others):
    """Side nm of the square compact lattice x; every other array (None
    allowed) must have x's shape."""
    if x.dim() != 2 or x.shape[0] != x.shape[1] or x.shape[0] < 3:
        raise ValueError("x must be a square lattice of side >= 3, got %s" % (tuple(x.shape),))
    for t, what in others:
        _shape(t, x.shape, what)
    return int(x.shape[0])


def learn_forward(x, r, a, w, hl, y, stream=None):
    """Network output of the learned relaxation on one compact lattice
    (dense float32 GPU arrays of side nm; a may be None)."""
    import torch
    f32 = torch.float32
    nm = _lattice(x, (r, "r"), (a, "a"), (y, "y"))
    _check_global(lib().homg_learn_forward(nm, hl, _ptr(x, f32), _ptr(r, f32),
                                           _ptr(a, f32) if a is not None else None,
                                           _ptr(_weights(w), f32), _ptr(y, f32), _stream(stream)))


def learn_grad(x, r, a, delta, w, hl, stream=None):
    """(dL/dw as a float64 GPU tensor of 576, E(delta - y), L) for one sample."""
    import torch
    f32 = torch.float32
    nm = _lattice(x, (r, "r"), (a, "a"), (delta, "delta"))
    g = torch.empty(SMOOTHER_WEIGHTS + 1, dtype=torch.float64, device="cuda")
    loss = ctypes.c_double()
    _check_global(lib().homg_learn_grad(nm, hl, _ptr(x, f32), _ptr(r, f32),
                                        _ptr(a, f32) if a is not None else None, _ptr(delta, f32),
                                        _ptr(_weights(w), f32), _ptr(g), ctypes.byref(loss), _stream(stream)))
    return g[:SMOOTHER_WEIGHTS], float(g[SMOOTHER_WEIGHTS]), loss.value


def learn_adam(theta, m1, m2, grad, t, lr, w_out, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch
    f32 = torch.float32
    for v, what in ((theta, "theta"), (m1, "m1"), (m2, "m2"), (grad, "grad"), (w_out, "w_out")):
        _shape(v, (SMOOTHER_WEIGHTS,), what)
    _check_global(lib().homg_learn_adam(_ptr(theta, f32), _ptr(m1, f32), _ptr(m2, f32), _ptr(grad), t, lr,
                                        beta1, beta2, eps, _ptr(w_out, f32), _stream(stream)))


def residual_noalloc(f, u, r, stream=None):
    """r = f - A u (Laplacian) and ||r|| / ||f|| with no handle and no device
    allocation (the library's static workspace); f, u, r dense float64 GPU
    arrays of the same cubic/square shape."""
    ndim = f.dim()
    n = int(f.shape[0])
    _shape(f, (n,) * ndim, "f")
    _shape(u, (n,) * ndim, "u")
    _shape(r, (n,) * ndim, "r")
    rel = ctypes.c_double()
    _check_global(lib().homg_residual_noalloc(ndim, n, _ptr(f), _ptr(u), _ptr(r), ctypes.byref(rel),
                                              _stream(stream)))
    return rel.value


class BatchSolver:
    """Many independent 2D Poisson problems advanced together (one launch per step for all)."""

    def __init__(self, sides, precision="fp32", omega=0.0, max_i=4, max_cycles=200):
        L = lib()
        opt = Options()
        L.homg_options_init(ctypes.byref(opt))
        opt.omega = omega
        opt.max_i = max_i
        opt.max_cycles = max_cycles
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.sides = [int(v) for v in sides]
        arr = (ctypes.c_int64 * len(self.sides))(*self.sides)
        h = ctypes.c_void_p()
        st = L.homg_batch_create(ctypes.byref(h), len(self.sides), arr, ctypes.byref(opt))
        if st != HOMG_OK:
            raise HomgError(st, L.homg_last_error(None).decode())
        self._h = h

    def _check(self, st):
        if st != HOMG_OK:
            raise HomgError(st, lib().homg_last_error(None).decode())

    def _check_arrays(self, fs, us):
        n = len(self.sides)
        if len(fs) != n or len(us) != n:
            raise ValueError("need one f and one u per problem")
        for i, side in enumerate(self.sides):
            _shape(fs[i], (side, side), "f[%d]" % i)
            _shape(us[i], (side, side), "u[%d]" % i)

    @staticmethod
    def _ptrs(ts):
        return (ctypes.c_void_p * len(ts))(*[_ptr(t).value for t in ts])

    def solve(self, fs, us, tol=1e-10, stream=None, raise_on_status=True):
        self._check_arrays(fs, us)
        n = len(self.sides)
        rel = (ctypes.c_double * n)()
        cyc = (ctypes.c_int * n)()
        sts = (ctypes.c_int * n)()
        st = lib().homg_batch_solve(self._h, self._ptrs(fs), self._ptrs(us), tol, _stream(stream), rel, cyc, sts)
        out = {"status": st, "relres": list(rel), "cycles": list(cyc), "statuses": list(sts)}
        if raise_on_status:
            self._check(st)
        return out

    def set_tile_rows(self, side, rows):
        self._check(lib().homg_batch_set_tile_rows(self._h, side, rows))

    def set_pass_iters(self, side, iters):
        self._check(lib().homg_batch_set_pass_iters(self._h, side, iters))

    def tune(self, fs, us, tol=1e-10, cache_path=None, stream=None):
        self._check_arrays(fs, us)
        self._check(lib().homg_batch_tune(self._h, self._ptrs(fs), self._ptrs(us), tol, _stream(stream),
                                          cache_path.encode() if cache_path else None))

    def close(self):
        if getattr(self, "_h", None):
            lib().homg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version():
    return lib().homg_version().decode()
