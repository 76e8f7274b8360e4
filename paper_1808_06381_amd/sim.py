"""Thin ctypes binding of libsim (include/sim.h).  Argument marshalling only:
every step of the simulation runs in the library's HIP kernels.  PyTorch is
used for streams and, optionally, device memory (SIM_DEVICE_PTR calls).

The functions keep the C names (sim_create, sim_step, sim_solve, sim_state,
...); ``Sim`` wraps a handle with numpy in / numpy out.  The library must be
built (``paper_1808_06381_amd.build``); loading fails loudly otherwise.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libsim.so")

SIM_OK = 0
SIM_DEVICE_PTR = 1
ERRORS = {-1: "SIM_EINVAL", -2: "SIM_ENOMEM", -3: "SIM_EDEVICE", -4: "SIM_ENOCONV",
          -5: "SIM_EBREAKDOWN", -6: "SIM_ECAPACITY", -7: "SIM_ENUMERIC", -8: "SIM_ENOTSUP"}
W_LAWS = {"gauss": 0, "poly2": 1}
POTENTIALS = {"gauss_core": 0, "soft": 1, "none": 2}
NOISE = {"fdt": 0, "paper": 1, "off": 2}
PRECOND = {"jacobi": 0, "none": 1, "ic0": 2, "learned": 3}

EXPORTED = ["sim_create", "sim_create_batch", "sim_step", "sim_solve", "sim_state",
            "sim_set_stream", "sim_load_precond", "sim_debug_pairs", "sim_debug_system",
            "sim_debug_set_gaussians", "sim_debug_block_system", "sim_profile_enable", "sim_profile_read",
            "sim_copy_probe", "sim_event_probe", "sim_structure_factor",
            "sim_structure_factor_noalloc",
            "sim_velocity_correlation", "sim_precond_weights",
            "sim_precond_config", "sim_precond_floor", "sim_train_step",
            "sim_precond_grad", "sim_debug_precond", "sim_graph_mode", "sim_graph_info",
            "sim_autotune", "sim_set_tuning", "sim_train_probe", "sim_precond_optimizer",
            "sim_destroy", "sim_strerror"]
MPNN_NPARAMS = 9893
MPNN_NPARAMS_BLOCK = 9962  # with the 3 x 3 heads of the block system


# CSR product variants of sim_tuning: (lanes per row, entries per lane loaded one
# pass ahead of the gathers; 0 = one at a time), or (0, entries per thread and
# pass) for the entry-parallel form, in the library's index order
CSR_VARIANTS = [(1, 0), (2, 0), (4, 0), (8, 0), (2, 2), (4, 1), (4, 2), (4, 3), (0, 2), (0, 3)]


class SimTuning(C.Structure):
    _fields_ = [("spmv_variant", C.c_int32), ("apply_variant", C.c_int32),
                ("spmv_us", C.c_float * len(CSR_VARIANTS)),
                ("apply_us", C.c_float * len(CSR_VARIANTS)),
                ("vec_variant", C.c_int32), ("vec_us", C.c_float * 2)]

    def as_dict(self):
        return dict(spmv_variant=self.spmv_variant, apply_variant=self.apply_variant,
                    spmv_us=list(self.spmv_us), apply_us=list(self.apply_us),
                    vec_variant=self.vec_variant, vec_us=list(self.vec_us))


class SimParams(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("box", C.c_double * 3),
        ("kT", C.c_double),
        ("gamma0", C.c_double),
        ("alpha", C.c_double),
        ("shear_rate", C.c_double),
        ("dt", C.c_double),
        ("rc", C.c_double),
        ("lambda_", C.c_double),
        ("u_amp", C.c_double),
        ("weight_law", C.c_int32),
        ("potential", C.c_int32),
        ("noise_mode", C.c_int32),
        ("precond", C.c_int32),
        ("spmv_fp32", C.c_int32),
        ("warm_start", C.c_int32),
        ("cg_maxit", C.c_int32),
        ("reserved0", C.c_int32),
        ("cg_tol", C.c_double),
        ("seed", C.c_uint64),
        ("stream", C.c_uint64),
        ("friction_par", C.c_double),
        ("friction_perp", C.c_double),
    ]


class SimStats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32 * 3),
        ("restarts", C.c_int32),
        ("relres", C.c_double * 3),
        ("nnz", C.c_int64),
        ("max_row", C.c_int32),
        ("fallback", C.c_int32),
        ("steps_done", C.c_int64),
        ("cg_iters_total", C.c_int64),
    ]

    def as_dict(self):
        return dict(iters=list(self.iters), restarts=self.restarts, relres=list(self.relres),
                    nnz=self.nnz, max_row=self.max_row, fallback=self.fallback,
                    steps_done=self.steps_done, cg_iters_total=self.cg_iters_total)


class SimMeta(C.Structure):
    _fields_ = [
        ("step", C.c_int64),
        ("time", C.c_double),
        ("le_offset", C.c_double),
        ("replicas", C.c_int32),
        ("reserved0", C.c_int32),
        ("n_total", C.c_int64),
    ]


class SimKernelProf(C.Structure):
    _fields_ = [
        ("name", C.c_char * 32),
        ("launches", C.c_int64),
        ("ms", C.c_double),
        ("bytes", C.c_double),
    ]


class SimError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().sim_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({msg})")


_lib = None


def lib():
    """Load libsim.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsim.so not built ({LIB_PATH}); run paper_1808_06381_amd.build")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.sim_create.argtypes = [P(SimParams), vp, P(vp)]
        L.sim_create_batch.argtypes = [P(SimParams), C.c_int32, vp, P(vp)]
        L.sim_step.argtypes = [vp, C.c_int32, P(SimStats)]
        L.sim_solve.argtypes = [vp, vp, vp, C.c_double, C.c_uint32, P(SimStats)]
        L.sim_state.argtypes = [vp, vp, vp, P(SimMeta), C.c_uint32]
        L.sim_structure_factor.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp,
                                           P(C.c_double)]
        L.sim_structure_factor_noalloc.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.sim_velocity_correlation.argtypes = [vp, C.c_double, C.c_int32, C.c_int32, vp, vp, vp,
                                               P(C.c_double)]
        L.sim_set_stream.argtypes = [vp, vp]
        L.sim_load_precond.argtypes = [vp, C.c_char_p]
        L.sim_debug_pairs.argtypes = [vp, vp, C.c_int64, P(C.c_int64)]
        L.sim_debug_system.argtypes = [vp, vp, vp, vp, C.c_int64, P(C.c_int64), vp, vp]
        L.sim_debug_block_system.argtypes = [vp, vp, vp, vp, C.c_int64, P(C.c_int64), vp, vp]
        L.sim_debug_set_gaussians.argtypes = [vp, vp, vp]
        L.sim_profile_enable.argtypes = [vp, C.c_int32]
        L.sim_profile_read.argtypes = [vp, P(SimKernelProf), C.c_int32, P(C.c_int32), C.c_int32]
        L.sim_copy_probe.argtypes = [vp, vp, C.c_int64, C.c_int32, vp, P(C.c_double)]
        L.sim_event_probe.argtypes = [vp, vp, C.c_int64, C.c_int32, vp, P(C.c_double),
                                      P(C.c_double)]
        L.sim_precond_weights.argtypes = [vp, vp, C.c_int64, C.c_int32]
        L.sim_precond_config.argtypes = [vp, C.c_int32, C.c_int32]
        L.sim_precond_floor.argtypes = [vp, C.c_double]
        L.sim_graph_mode.argtypes = [vp, C.c_int32]
        L.sim_train_probe.argtypes = [vp, C.c_double, C.c_uint64, C.c_uint64, C.c_int32,
                                      P(C.c_double)]
        L.sim_precond_optimizer.argtypes = [vp, vp, vp, C.c_int64, P(C.c_int32), C.c_int32]
        L.sim_graph_info.argtypes = [vp, P(C.c_int64), P(C.c_int64)]
        L.sim_autotune.argtypes = [vp, C.c_int32, P(SimTuning)]
        L.sim_set_tuning.argtypes = [vp, P(SimTuning)]
        L.sim_train_step.argtypes = [vp, C.c_double, P(C.c_double)]
        L.sim_precond_grad.argtypes = [vp, vp, C.c_int64]
        L.sim_debug_precond.argtypes = [vp, vp, vp, vp, C.c_int64, P(C.c_int64), vp]
        L.sim_destroy.argtypes = [vp]
        L.sim_destroy.restype = None
        L.sim_strerror.argtypes = [C.c_int]
        L.sim_strerror.restype = C.c_char_p
        for f in EXPORTED:
            if f not in ("sim_destroy", "sim_strerror"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def make_params(cfg, tol=None, maxit=None, precond=None, spmv_fp32=None):
    """Parameter dict (paper_1808_06381_amd.inputs vocabulary) -> SimParams."""
    p = SimParams()
    p.n = int(cfg["n"])
    for k in range(3):
        p.box[k] = float(cfg["box"][k])
    p.kT = float(cfg["kT"])
    p.gamma0 = float(cfg["gamma0"])
    p.alpha = float(cfg["alpha"])
    p.shear_rate = float(cfg["shear_rate"])
    p.dt = float(cfg["dt"])
    p.rc = float(cfg["rc"])
    p.lambda_ = float(cfg.get("lam", 1.0))
    p.u_amp = float(cfg.get("u_amp", 0.0))
    p.weight_law = W_LAWS[cfg.get("weight_law", "poly2")]
    p.potential = POTENTIALS[cfg.get("potential", "soft")]
    p.noise_mode = NOISE[cfg.get("noise", "fdt")]
    p.precond = PRECOND[precond or cfg.get("precond", "jacobi")]
    p.spmv_fp32 = int(cfg.get("spmv_fp32", 0) if spmv_fp32 is None else spmv_fp32)
    p.warm_start = int(cfg.get("warm_start", 0))
    p.friction_par = float(cfg.get("friction_par", 1.0))
    p.friction_perp = float(cfg.get("friction_perp", 1.0))
    p.cg_maxit = int(maxit or cfg.get("cg_maxit", 10000))
    p.cg_tol = float(tol or cfg.get("cg_tol", 1e-10))
    p.seed = int(cfg.get("seed", 0)) & (2**64 - 1)
    p.stream = int(cfg.get("stream", 0)) & (2**64 - 1)
    return p


def _check(code, where):
    if code != SIM_OK:
        raise SimError(code, where)


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


class Sim:
    """One handle: a single box (cfg dict) or a batch (list of cfg dicts)."""

    def __init__(self, cfg, pos0, tol=None, maxit=None, precond=None, spmv_fp32=None,
                 stream=None):
        L = lib()
        cfgs = cfg if isinstance(cfg, (list, tuple)) else [cfg]
        self.cfgs = list(cfgs)
        arr = (SimParams * len(cfgs))(*[make_params(c, tol, maxit, precond, spmv_fp32)
                                        for c in cfgs])
        pos0 = np.ascontiguousarray(pos0, dtype=np.float64).reshape(-1, 3)
        self.n_total = sum(int(c["n"]) for c in cfgs)
        self.replicas = len(cfgs)
        # friction other than 1 along or across the line of centres (0 stands
        # for 1): the library solves the block system (3 x 3 blocks)
        self.block = any(float(c.get(k, 1.0)) not in (0.0, 1.0)
                         for c in cfgs for k in ("friction_par", "friction_perp"))
        self.nparams = MPNN_NPARAMS_BLOCK if self.block else MPNN_NPARAMS
        if pos0.shape[0] != self.n_total:
            raise ValueError("pos0 rows != total particles")
        h = C.c_void_p()
        _check(L.sim_create_batch(arr, len(cfgs), _ptr(pos0), C.byref(h)), "sim_create_batch")
        self.h = h
        if stream is not None:
            self.set_stream(stream)

    def close(self):
        if getattr(self, "h", None):
            lib().sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, a raw hipStream_t int, or None."""
        raw = getattr(stream, "cuda_stream", stream)
        _check(lib().sim_set_stream(self.h, C.c_void_p(raw or 0)), "sim_set_stream")

    def step(self, nsteps=1):
        st = SimStats()
        _check(lib().sim_step(self.h, int(nsteps), C.byref(st)), "sim_step")
        return st.as_dict()

    def solve(self, b, tol=0.0):
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(self.n_total, 3)
        v = np.zeros_like(b)
        st = SimStats()
        _check(lib().sim_solve(self.h, _ptr(b), _ptr(v), float(tol), 0, C.byref(st)), "sim_solve")
        return v, st.as_dict()

    def solve_device(self, b, v, tol=0.0):
        """b, v: contiguous float64 torch tensors on the library's device."""
        st = SimStats()
        _check(lib().sim_solve(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(v.data_ptr()),
                               float(tol), SIM_DEVICE_PTR, C.byref(st)), "sim_solve")
        return st.as_dict()

    def state(self):
        pos = np.zeros((self.n_total, 3))
        vel = np.zeros((self.n_total, 3))
        meta = SimMeta()
        _check(lib().sim_state(self.h, _ptr(pos), _ptr(vel), C.byref(meta), 0), "sim_state")
        return pos, vel, dict(step=meta.step, time=meta.time, le_offset=meta.le_offset,
                              replicas=meta.replicas, n_total=meta.n_total)

    def structure_factor(self, nx, my_max, mz=0, timed=False):
        """S(q) of every replica on the Lees-Edwards grid: array (replicas,
        nx, 2 my_max + 1), [r, mx, my + my_max]; with timed=True also the
        contraction kernel's duration in ms."""
        ny = 2 * int(my_max) + 1
        # sized for valid arguments; the library rejects the others
        out = np.zeros((self.replicas, max(int(nx), 0), max(ny, 0)))
        ms = C.c_double()
        _check(lib().sim_structure_factor(self.h, int(nx), int(my_max), int(mz), _ptr(out),
                                          C.byref(ms) if timed else None),
               "sim_structure_factor")
        return (out, ms.value) if timed else out

    def structure_factor_noalloc(self, nx, my_max, out, mz=0):
        """S(q) as structure_factor, written into `out`, a contiguous float64
        torch tensor on the library's device of shape (replicas, nx,
        2 my_max + 1); the library allocates nothing for the call."""
        ny = 2 * int(my_max) + 1
        if tuple(out.shape) != (self.replicas, int(nx), ny) or not out.is_contiguous():
            raise ValueError("out must be a contiguous (replicas, nx, 2 my_max + 1) tensor")
        _check(lib().sim_structure_factor_noalloc(self.h, int(nx), int(my_max), int(mz),
                                                  C.c_void_p(out.data_ptr())),
               "sim_structure_factor_noalloc")
        return out

    def velocity_correlation(self, r_max, nbins, flow=True, timed=False):
        """Velocity cross-correlation of the last committed step (the
        configuration the velocities were solved at): per replica and
        distance bin the sum of u_i . u_j and the count over unordered pairs
        with r < r_max, and sum |u|^2; u relative to the Couette flow when
        flow is set.  Returns (sum (replicas, nbins), count (replicas,
        nbins), u2 (replicas,)), with timed=True also the pair kernel's
        duration in ms."""
        nb = max(int(nbins), 0)
        s = np.zeros((self.replicas, nb))
        c = np.zeros((self.replicas, nb), dtype=np.int64)
        u2 = np.zeros(self.replicas)
        ms = C.c_double()
        _check(lib().sim_velocity_correlation(self.h, float(r_max), int(nbins), int(bool(flow)),
                                              _ptr(s), _ptr(c), _ptr(u2),
                                              C.byref(ms) if timed else None),
               "sim_velocity_correlation")
        return (s, c, u2, ms.value) if timed else (s, c, u2)

    def pairs(self):
        """Unordered pairs as an int64 (m, 3) array of (replica, i, j), sorted."""
        cnt = C.c_int64()
        rc = lib().sim_debug_pairs(self.h, None, 0, C.byref(cnt))
        if rc not in (SIM_OK, -6):
            _check(rc, "sim_debug_pairs")
        out = np.zeros((max(cnt.value, 1), 3), dtype=np.int64)
        _check(lib().sim_debug_pairs(self.h, _ptr(out), cnt.value, C.byref(cnt)), "sim_debug_pairs")
        out = out[:cnt.value]
        order = np.lexsort((out[:, 2], out[:, 1], out[:, 0]))
        return out[order]

    def system(self):
        """(rows, cols, vals, diag, rhs) of the current system, global original ids."""
        cnt = C.c_int64()
        rc = lib().sim_debug_system(self.h, None, None, None, 0, C.byref(cnt), None, None)
        if rc not in (SIM_OK, -6):
            _check(rc, "sim_debug_system")
        m = max(cnt.value, 1)
        rows = np.zeros(m, dtype=np.int64)
        cols = np.zeros(m, dtype=np.int64)
        vals = np.zeros(m)
        diag = np.zeros(self.n_total)
        rhs = np.zeros((self.n_total, 3))
        _check(lib().sim_debug_system(self.h, _ptr(rows), _ptr(cols), _ptr(vals), cnt.value,
                                      C.byref(cnt), _ptr(diag), _ptr(rhs)), "sim_debug_system")
        k = cnt.value
        return rows[:k], cols[:k], vals[:k], diag, rhs

    def block_system(self):
        """(rows, cols, vals (m, 3, 3), diag (n, 3, 3), rhs) of the current
        block system (anisotropic friction), global original ids."""
        cnt = C.c_int64()
        rc = lib().sim_debug_block_system(self.h, None, None, None, 0, C.byref(cnt), None, None)
        if rc not in (SIM_OK, -6):
            _check(rc, "sim_debug_block_system")
        m = max(cnt.value, 1)
        rows = np.zeros(m, dtype=np.int64)
        cols = np.zeros(m, dtype=np.int64)
        vals = np.zeros((m, 3, 3))
        diag = np.zeros((self.n_total, 3, 3))
        rhs = np.zeros((self.n_total, 3))
        _check(lib().sim_debug_block_system(self.h, _ptr(rows), _ptr(cols), _ptr(vals), cnt.value,
                                            C.byref(cnt), _ptr(diag), _ptr(rhs)),
               "sim_debug_block_system")
        k = cnt.value
        return rows[:k], cols[:k], vals[:k], diag, rhs

    def set_gaussians(self, xi=None, eta=None):
        if xi is None and eta is None:
            _check(lib().sim_debug_set_gaussians(self.h, None, None), "sim_debug_set_gaussians")
            return
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        _check(lib().sim_debug_set_gaussians(self.h, _ptr(xi), _ptr(eta)),
               "sim_debug_set_gaussians")

    def profile_enable(self, sample_every):
        _check(lib().sim_profile_enable(self.h, int(sample_every)), "sim_profile_enable")

    def profile_read(self, reset=True):
        """{kernel: dict(launches, ms, bytes)} of the timing probe."""
        arr = (SimKernelProf * 8)()
        cnt = C.c_int32()
        _check(lib().sim_profile_read(self.h, arr, 8, C.byref(cnt), int(reset)), "sim_profile_read")
        return {arr[k].name.decode(): dict(launches=arr[k].launches, ms=arr[k].ms,
                                           bytes=arr[k].bytes) for k in range(cnt.value)}

    def train_probe(self, lr, seed, index, norm="2"):
        """One Adam step on a white-noise probe z (x* = z, b = A z) with the loss
        in the Euclidean ("2") or the A-norm ("A"); returns the loss before the
        update."""
        if norm not in ("A", "2"):
            raise ValueError("norm must be 'A' or '2'")
        loss = C.c_double()
        _check(lib().sim_train_probe(self.h, float(lr), int(seed) & (2**64 - 1),
                                     int(index) & (2**64 - 1), 1 if norm == "2" else 0,
                                     C.byref(loss)), "sim_train_probe")
        return loss.value

    def get_optimizer(self):
        m1 = np.zeros(self.nparams, dtype=np.float32)
        m2 = np.zeros(self.nparams, dtype=np.float32)
        t = C.c_int32()
        _check(lib().sim_precond_optimizer(self.h, _ptr(m1), _ptr(m2), m1.size, C.byref(t), 0),
               "sim_precond_optimizer")
        return m1, m2, t.value

    def set_optimizer(self, state):
        m1, m2, t = state
        m1 = np.ascontiguousarray(m1, dtype=np.float32)
        m2 = np.ascontiguousarray(m2, dtype=np.float32)
        tt = C.c_int32(int(t))
        _check(lib().sim_precond_optimizer(self.h, _ptr(m1), _ptr(m2), m1.size, C.byref(tt), 1),
               "sim_precond_optimizer")

    def graph_mode(self, on=True):
        _check(lib().sim_graph_mode(self.h, int(bool(on))), "sim_graph_mode")

    def graph_info(self):
        c, r = C.c_int64(), C.c_int64()
        _check(lib().sim_graph_info(self.h, C.byref(c), C.byref(r)), "sim_graph_info")
        return dict(captures=c.value, replays=r.value)

    def autotune(self, reps=20):
        t = SimTuning()
        _check(lib().sim_autotune(self.h, int(reps), C.byref(t)), "sim_autotune")
        return t.as_dict()

    def set_tuning(self, spmv_variant=8, apply_variant=8, vec_variant=0):
        """Fix the CSR product variants (indices into CSR_VARIANTS) and the
        vector kernel's form (0 ordinary, 1 nontemporal accesses)."""
        t = SimTuning()
        t.spmv_variant, t.apply_variant = int(spmv_variant), int(apply_variant)
        t.vec_variant = int(vec_variant)
        _check(lib().sim_set_tuning(self.h, C.byref(t)), "sim_set_tuning")

    def set_weights(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        _check(lib().sim_precond_weights(self.h, _ptr(theta), theta.size, 1), "sim_precond_weights")

    def get_weights(self):
        theta = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().sim_precond_weights(self.h, _ptr(theta), theta.size, 0), "sim_precond_weights")
        return theta

    def precond_config(self, round_act=True, learned_maxit=0):
        _check(lib().sim_precond_config(self.h, int(bool(round_act)), int(learned_maxit)),
               "sim_precond_config")

    def precond_floor(self, lam_floor=0.3):
        """Floor added to the learned diagonal head (default 0.3)."""
        _check(lib().sim_precond_floor(self.h, float(lam_floor)), "sim_precond_floor")

    def train_step(self, lr):
        loss = C.c_double()
        _check(lib().sim_train_step(self.h, float(lr), C.byref(loss)), "sim_train_step")
        return loss.value

    def precond_grad(self):
        g = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().sim_precond_grad(self.h, _ptr(g), g.size), "sim_precond_grad")
        return g

    def precond_matrix(self):
        """(rows, cols, vals, diag) of the preconditioner at the current
        positions: the learned M^-1, or L's strictly lower triangle and diagonal
        for IC(0) (unused slots dropped).  Block handles: vals (nnz, 3, 3) and
        diag (n, 3, 3), the blocks of the learned M^-1."""
        cnt = C.c_int64()
        rc = lib().sim_debug_precond(self.h, None, None, None, 0, C.byref(cnt), None)
        if rc not in (SIM_OK, -6):
            _check(rc, "sim_debug_precond")
        m = max(cnt.value, 1)
        rows = np.zeros(m, dtype=np.int64)
        cols = np.zeros(m, dtype=np.int64)
        shape = (3, 3) if self.block else ()
        vals = np.zeros((m,) + shape)
        mdiag = np.zeros((self.n_total,) + shape)
        _check(lib().sim_debug_precond(self.h, _ptr(rows), _ptr(cols), _ptr(vals), cnt.value,
                                       C.byref(cnt), _ptr(mdiag)), "sim_debug_precond")
        k = cnt.value
        keep = rows[:k] >= 0
        return rows[:k][keep], cols[:k][keep], vals[:k][keep], mdiag

    def load_precond(self, path):
        _check(lib().sim_load_precond(self.h, path.encode()), "sim_load_precond")


def event_probe(src, dst, reps=64, stream=None):
    """(ms per copy in a chain between one event pair, ms per copy each
    between its own launch-bound event pair): the difference is what the
    kernel timing probe's events add to a timed launch."""
    chain, each = C.c_double(), C.c_double()
    raw = getattr(stream, "cuda_stream", stream) or 0
    nbytes = src.numel() * src.element_size()
    _check(lib().sim_event_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                                 int(reps), C.c_void_p(raw), C.byref(chain), C.byref(each)),
           "sim_event_probe")
    return chain.value, each.value


def copy_probe(src, dst, reps=20, stream=None):
    """Mean ms of one device copy src -> dst (torch tensors, same byte size)."""
    ms = C.c_double()
    raw = getattr(stream, "cuda_stream", stream) or 0
    nbytes = src.numel() * src.element_size()
    _check(lib().sim_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                                int(reps), C.c_void_p(raw), C.byref(ms)), "sim_copy_probe")
    return ms.value
