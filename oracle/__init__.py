"""ctypes binding of the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the GPU library; the only thing both sides take from one place is
the seeded input generator module, which holds none of the method's
arithmetic.

Parameters arrive as a plain dict (see ``paper_1808_06381_amd.inputs``):
    n, box, kT, gamma0, alpha, shear_rate, dt, rc, lam, u_amp,
    weight_law ('gauss' | 'poly2'), potential ('gauss_core' | 'soft' | 'none'),
    noise ('fdt' | 'paper' | 'off'), seed, stream
Arrays are numpy, particles in original id order, n x 3 row-major.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

W_LAWS = {"gauss": 0, "poly2": 1}
POTENTIALS = {"gauss_core": 0, "soft": 1, "none": 2}
NOISE = {"fdt": 0, "paper": 1, "off": 2}
PRECOND = {"jacobi": 0, "none": 1, "ic0": 2, "given": 3}
STATUS = {0: "ok", -2: "no memory", -4: "no convergence", -5: "breakdown"}


class OrcParams(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("box", C.c_double * 3),
        ("kT", C.c_double),
        ("gamma0", C.c_double),
        ("alpha", C.c_double),
        ("shear_rate", C.c_double),
        ("dt", C.c_double),
        ("rc", C.c_double),
        ("lam", C.c_double),
        ("u_amp", C.c_double),
        ("weight_law", C.c_int32),
        ("potential", C.c_int32),
        ("noise_mode", C.c_int32),
        ("pad0", C.c_int32),
        ("seed", C.c_uint64),
        ("stream", C.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # build on first use (CPU only, seconds)

            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        d_p = P(C.c_double)
        i64_p = P(C.c_int64)
        u64_p = P(C.c_uint64)
        pp = P(OrcParams)
        L.orc_philox4x64_10.argtypes = [u64_p, u64_p, u64_p]
        L.orc_gauss4.argtypes = [pp, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, d_p]
        L.orc_le_offset.argtypes = [pp, C.c_int64]
        L.orc_le_offset.restype = C.c_double
        L.orc_separation.argtypes = [pp, C.c_double, d_p, d_p, d_p]
        L.orc_separation.restype = C.c_int
        for f in (L.orc_pairs_brute, L.orc_pairs_cells):
            f.argtypes = [pp, C.c_double, d_p, C.c_int64, i64_p]
            f.restype = C.c_int64
        L.orc_count_pairs.argtypes = [pp, C.c_int64, d_p]
        L.orc_count_pairs.restype = C.c_int64
        L.orc_build_system.argtypes = [pp, C.c_int64, d_p, d_p, d_p, C.c_int64, i64_p, i64_p,
                                       d_p, d_p, d_p, d_p]
        L.orc_build_system.restype = C.c_int64
        L.orc_spmv3.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, d_p, d_p]
        L.orc_pcg.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, d_p, d_p, C.c_double, C.c_int,
                              C.c_int, i64_p, i64_p, d_p, d_p, P(C.c_int), d_p]
        L.orc_pcg.restype = C.c_int
        L.orc_ic0.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, C.c_int64, i64_p, i64_p, d_p]
        L.orc_ic0.restype = C.c_int64
        L.orc_step.argtypes = [pp, C.c_int64, d_p, d_p, C.c_double, C.c_int, C.c_int, P(C.c_int)]
        L.orc_step.restype = C.c_int
        L.orc_wrap.argtypes = [pp, C.c_int64, d_p]
        L.orc_build_block_system.argtypes = [pp, C.c_double, C.c_double, C.c_int64, d_p,
                                             C.c_int64, i64_p, i64_p, d_p, d_p, d_p]
        L.orc_build_block_system.restype = C.c_int64
        L.orc_block_pcg.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, d_p, d_p, C.c_double,
                                    C.c_int, P(C.c_int)]
        L.orc_block_pcg.restype = C.c_int
        L.orc_step_block.argtypes = [pp, C.c_double, C.c_double, C.c_int64, d_p, d_p,
                                     C.c_double, C.c_int, P(C.c_int)]
        L.orc_step_block.restype = C.c_int
        L.orc_velocity_correlation.argtypes = [pp, C.c_double, d_p, d_p, C.c_double, C.c_int32,
                                               C.c_int32, C.c_int32, d_p, i64_p, d_p]
        L.orc_velocity_correlation.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        f_p = P(C.c_float)
        L.orc_mpnn_nparams.restype = C.c_int64
        L.orc_bf16.argtypes = [C.c_float]
        L.orc_bf16.restype = C.c_double
        L.orc_mpnn_set_bf16.argtypes = [C.c_int]
        L.orc_mpnn_forward.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, d_p, C.c_double, f_p,
                                       d_p, d_p]
        L.orc_mpnn_forward.restype = C.c_int
        L.orc_mpnn_loss_grad.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, d_p, C.c_double, f_p,
                                         d_p, d_p, d_p]
        L.orc_mpnn_loss_grad.restype = C.c_double
        L.orc_mpnn_loss_grad_norm.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, d_p, C.c_double,
                                              f_p, d_p, d_p, C.c_int, d_p]
        L.orc_mpnn_loss_grad_norm.restype = C.c_double
        L.orc_mpnn_block_nparams.restype = C.c_int64
        L.orc_mpnn_block_forward.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, d_p, C.c_double,
                                             f_p, d_p, d_p]
        L.orc_mpnn_block_forward.restype = C.c_int
        L.orc_mpnn_block_loss_grad.argtypes = [C.c_int64, i64_p, i64_p, d_p, d_p, d_p,
                                               C.c_double, f_p, d_p, d_p, C.c_int, d_p]
        L.orc_mpnn_block_loss_grad.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def set_threads(n):
    """OpenMP threads of the oracle's row-parallel loops (1: sequential);
    results are the same bits with any count.  Returns the count in force."""
    lib().orc_set_threads(int(n))
    return lib().orc_get_threads()


def make_params(cfg):
    """dict -> OrcParams"""
    p = OrcParams()
    p.n = int(cfg["n"])
    for k in range(3):
        p.box[k] = float(cfg["box"][k])
    p.kT = float(cfg["kT"])
    p.gamma0 = float(cfg["gamma0"])
    p.alpha = float(cfg["alpha"])
    p.shear_rate = float(cfg["shear_rate"])
    p.dt = float(cfg["dt"])
    p.rc = float(cfg["rc"])
    p.lam = float(cfg.get("lam", 1.0))
    p.u_amp = float(cfg.get("u_amp", 0.0))
    p.weight_law = W_LAWS[cfg.get("weight_law", "poly2")]
    p.potential = POTENTIALS[cfg.get("potential", "soft")]
    p.noise_mode = NOISE[cfg.get("noise", "fdt")]
    p.seed = int(cfg.get("seed", 0)) & (2**64 - 1)
    p.stream = int(cfg.get("stream", 0)) & (2**64 - 1)
    return p


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    u64 = C.POINTER(C.c_uint64)
    lib().orc_philox4x64_10(c.ctypes.data_as(u64), k.ctypes.data_as(u64), out.ctypes.data_as(u64))
    return out


def gauss4(cfg, step, tag, a, b):
    p = make_params(cfg)
    g = np.zeros(4)
    lib().orc_gauss4(C.byref(p), step, tag, a, b, _dp(g))
    return g


def le_offset(cfg, step):
    return lib().orc_le_offset(C.byref(make_params(cfg)), int(step))


def separation(cfg, delta, ri, rj):
    p = make_params(cfg)
    ri = _f64(ri)
    rj = _f64(rj)
    d = np.zeros(3)
    s = lib().orc_separation(C.byref(p), float(delta), _dp(ri), _dp(rj), _dp(d))
    return d, s


def pairs(cfg, pos, delta=0.0, method="brute"):
    """Unordered pairs (i < j), sorted, as an int64 array of shape (m, 2)."""
    p = make_params(cfg)
    pos = _f64(pos, (-1, 3))
    f = lib().orc_pairs_brute if method == "brute" else lib().orc_pairs_cells
    m = f(C.byref(p), float(delta), _dp(pos), 0, None)
    if m < 0:
        raise MemoryError("oracle pair search failed")
    out = np.zeros((max(m, 1), 2), dtype=np.int64)
    f(C.byref(p), float(delta), _dp(pos), m, _ip(out))
    return out[:m]


def build_system(cfg, pos, step=0, xi=None, eta=None):
    """Friction system at step `step`; returns dict(rowptr, col, val, diag, rhs, fcons)."""
    p = make_params(cfg)
    n = p.n
    pos = _f64(pos, (n, 3))
    m = lib().orc_count_pairs(C.byref(p), int(step), _dp(pos))
    cap = 2 * m
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(cap, 1), dtype=np.int64)
    val = np.zeros(max(cap, 1))
    diag = np.zeros(n)
    rhs = np.zeros((n, 3))
    fcons = np.zeros((n, 3))
    xi = None if xi is None else _f64(xi, (n, 3))
    eta = None if eta is None else _f64(eta, (m, 3))
    nnz = lib().orc_build_system(C.byref(p), int(step), _dp(pos), _dp(xi), _dp(eta), cap,
                                 _ip(rowptr), _ip(col), _dp(val), _dp(diag), _dp(rhs),
                                 _dp(fcons))
    if nnz < 0:
        raise MemoryError("oracle system build failed")
    return dict(rowptr=rowptr, col=col[:nnz], val=val[:nnz], diag=diag, rhs=rhs, fcons=fcons,
                npairs=m)


def dense(sys_):
    """Dense A (n x n) from a build_system result (test helper)."""
    n = sys_["diag"].shape[0]
    A = np.diag(sys_["diag"]).astype(np.float64)
    rp = sys_["rowptr"]
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            A[i, sys_["col"][k]] += sys_["val"][k]
    return A


def spmv3(sys_, x):
    n = sys_["diag"].shape[0]
    x = _f64(x, (n, 3))
    y = np.zeros((n, 3))
    lib().orc_spmv3(n, _ip(sys_["rowptr"]), _ip(sys_["col"]), _dp(sys_["val"]),
                    _dp(sys_["diag"]), _dp(x), _dp(y))
    return y


def pcg(sys_, rhs=None, tol=1e-10, maxit=10000, precond="jacobi", x0=None, m=None):
    """Solve (A (x) I3) x = rhs; returns (x, iters[3], relres[3]).

    precond 'given' applies z = M r with m = dict(rowptr, col, val, diag)."""
    n = sys_["diag"].shape[0]
    rhs = _f64(sys_["rhs"] if rhs is None else rhs, (n, 3))
    x = np.zeros((n, 3)) if x0 is None else _f64(x0, (n, 3)).copy()
    iters = (C.c_int * 3)()
    rel = np.zeros(3)
    mr = mc = mv = md = None
    if precond == "given":
        mr, mc = m["rowptr"].astype(np.int64), m["col"].astype(np.int64)
        mv, md = _f64(m["val"]), _f64(m["diag"])
    st = lib().orc_pcg(n, _ip(sys_["rowptr"]), _ip(sys_["col"]), _dp(sys_["val"]),
                       _dp(sys_["diag"]), _dp(rhs), _dp(x), float(tol), int(maxit),
                       PRECOND[precond], _ip(mr), _ip(mc), _dp(mv), _dp(md), iters, _dp(rel))
    if st != 0:
        raise RuntimeError("oracle pcg: " + STATUS.get(st, str(st)))
    return x, list(iters), rel


def ic0(sys_):
    """IC(0) factor L of A in the system's row order: (lrow, lcol, lval) CSR,
    per row the strictly lower entries (ascending column) then L_ii."""
    n = sys_["diag"].shape[0]
    cap = n + len(sys_["col"]) // 2 + 1
    lrow = np.zeros(n + 1, dtype=np.int64)
    lcol = np.zeros(cap, dtype=np.int64)
    lval = np.zeros(cap)
    cnt = lib().orc_ic0(n, _ip(sys_["rowptr"]), _ip(sys_["col"]), _dp(sys_["val"]),
                        _dp(sys_["diag"]), cap, _ip(lrow), _ip(lcol), _dp(lval))
    if cnt < 0 or cnt > cap:
        raise RuntimeError("oracle ic0: " + STATUS.get(int(cnt), str(cnt)))
    return lrow, lcol[:cnt], lval[:cnt]


def step(cfg, pos, step_index, tol=1e-10, maxit=10000, precond="jacobi"):
    """One step; returns (new_pos, vel, iters)."""
    p = make_params(cfg)
    pos = _f64(pos, (p.n, 3)).copy()
    vel = np.zeros((p.n, 3))
    iters = (C.c_int * 3)()
    st = lib().orc_step(C.byref(p), int(step_index), _dp(pos), _dp(vel), float(tol), int(maxit),
                        PRECOND[precond], iters)
    if st != 0:
        raise RuntimeError("oracle step: " + STATUS.get(st, str(st)))
    return pos, vel, list(iters)


def run(cfg, pos, nsteps, first_step=0, tol=1e-10, maxit=10000, precond="jacobi"):
    """nsteps steps; returns (pos, last_vel, iteration counts per step)."""
    pos = _f64(pos, (-1, 3)).copy()
    vel = None
    its = []
    for k in range(nsteps):
        pos, vel, it = step(cfg, pos, first_step + k, tol, maxit, precond)
        its.append(it)
    return pos, vel, its


def wrap(cfg, pos, step_after):
    p = make_params(cfg)
    pos = _f64(pos, (p.n, 3)).copy()
    lib().orc_wrap(C.byref(p), int(step_after), _dp(pos))
    return pos


# ---- learned preconditioner ---------------------------------------------------

def build_block_system(cfg, pos, a_par, a_perp, step=0):
    """Anisotropic friction system (block.c): dict(rowptr, col, bval (m, 3, 3),
    bdiag (n, 3, 3), rhs (n, 3)), original ids, rows' entries in pair order."""
    p = make_params(cfg)
    n = p.n
    pos = _f64(pos, (-1, 3))
    np_ = lib().orc_count_pairs(C.byref(p), int(step), _dp(pos))
    cap = max(2 * np_, 1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(cap, dtype=np.int64)
    bval = np.zeros((cap, 3, 3))
    bdiag = np.zeros((n, 3, 3))
    rhs = np.zeros((n, 3))
    m = lib().orc_build_block_system(C.byref(p), float(a_par), float(a_perp), int(step), _dp(pos),
                                     cap, _ip(rowptr), _ip(col), _dp(bval), _dp(bdiag), _dp(rhs))
    if m < 0:
        raise MemoryError("oracle block system failed")
    return dict(rowptr=rowptr, col=col[:m], bval=bval[:m], bdiag=bdiag, rhs=rhs)


def block_dense(sys_):
    """the 3n x 3n matrix of a block system"""
    n = len(sys_["bdiag"])
    A = np.zeros((3 * n, 3 * n))
    for i in range(n):
        A[3 * i:3 * i + 3, 3 * i:3 * i + 3] = sys_["bdiag"][i]
        for e in range(sys_["rowptr"][i], sys_["rowptr"][i + 1]):
            j = sys_["col"][e]
            A[3 * i:3 * i + 3, 3 * j:3 * j + 3] = sys_["bval"][e]
    return A


def block_pcg(sys_, rhs=None, tol=1e-12, maxit=20000):
    n = len(sys_["bdiag"])
    b = _f64(sys_["rhs"] if rhs is None else rhs, (n, 3))
    x = np.zeros((n, 3))
    it = C.c_int(0)
    rc = lib().orc_block_pcg(n, _ip(sys_["rowptr"]), _ip(np.ascontiguousarray(sys_["col"])),
                             _dp(np.ascontiguousarray(sys_["bval"])), _dp(sys_["bdiag"]), _dp(b),
                             _dp(x), float(tol), int(maxit), C.byref(it))
    if rc:
        raise RuntimeError(f"oracle block PCG status {rc}")
    return x, it.value


def step_block(cfg, pos, step_index, a_par, a_perp, tol=1e-10, maxit=20000):
    """one step with anisotropic friction; returns (new positions, velocities, iterations)"""
    p = make_params(cfg)
    pos = _f64(pos, (-1, 3)).copy()
    vel = np.zeros_like(pos)
    it = C.c_int(0)
    rc = lib().orc_step_block(C.byref(p), float(a_par), float(a_perp), int(step_index), _dp(pos),
                              _dp(vel), float(tol), int(maxit), C.byref(it))
    if rc:
        raise RuntimeError(f"oracle block step status {rc}")
    return pos, vel, it.value


def velocity_correlation(cfg, delta, pos, vel, r_max, nbins, flow=True, cells=None):
    """Pair sums of u_i . u_j, pair counts (unordered pairs) per distance bin
    and sum_c |u_c|^2 (vv.c).  cells: cell-list pair search (default for
    n > 2048), else brute force."""
    p = make_params(cfg)
    pos = _f64(pos, (-1, 3))
    vel = _f64(vel, (-1, 3))
    if cells is None:
        cells = p.n > 2048
    s = np.zeros(nbins)
    c = np.zeros(nbins, dtype=np.int64)
    u2 = np.zeros(1)
    rc = lib().orc_velocity_correlation(C.byref(p), float(delta), _dp(pos), _dp(vel),
                                        float(r_max), int(nbins), int(bool(flow)), int(bool(cells)),
                                        _dp(s), _ip(c), _dp(u2))
    if rc == -1:
        raise ValueError("bad velocity-correlation arguments")
    if rc:
        raise MemoryError("oracle velocity correlation failed")
    return s, c, float(u2[0])


def mpnn_nparams():
    return int(lib().orc_mpnn_nparams())


def bf16(x):
    return lib().orc_bf16(float(x))


def mpnn_set_bf16(on):
    lib().orc_mpnn_set_bf16(1 if on else 0)


def edge_r(cfg, pos, sys_, step=0):
    """r_ij / rc per CSR entry of a build_system or build_block_system result
    (oracle geometry)."""
    delta = le_offset(cfg, step)
    n = len(sys_["rowptr"]) - 1
    out = np.zeros(len(sys_["col"]))
    rp = sys_["rowptr"]
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            d, _ = separation(cfg, delta, pos[i], pos[sys_["col"][k]])
            out[k] = np.sqrt(float(d @ d)) / cfg["rc"]
    return out


def _theta(theta):
    t = np.ascontiguousarray(theta, dtype=np.float32)
    assert t.shape == (mpnn_nparams(),)
    return t, t.ctypes.data_as(C.POINTER(C.c_float))


def mpnn_forward(sys_, er, alpha, theta):
    """M^-1 of the learned preconditioner: (mdiag[n], moff[nnz]) in A's pattern."""
    n = sys_["diag"].shape[0]
    t, tp = _theta(theta)
    mdiag = np.zeros(n)
    moff = np.zeros(max(len(sys_["col"]), 1))
    er = np.ascontiguousarray(er, dtype=np.float64)
    rc = lib().orc_mpnn_forward(n, _ip(sys_["rowptr"]), _ip(sys_["col"]), _dp(sys_["val"]),
                                _dp(sys_["diag"]), _dp(er), float(alpha), tp, _dp(mdiag),
                                _dp(moff))
    if rc != 0:
        raise RuntimeError("oracle mpnn forward failed")
    return mdiag, moff[:len(sys_["col"])]


def mpnn_loss_grad(sys_, er, alpha, theta, b, xstar, grad=True, norm="A"):
    """Loss ||M^-1 b - x*||^2 / ||x*||^2 in the A-norm (norm="A") or the
    Euclidean norm (norm="2") and its gradient (float64 array)."""
    n = sys_["diag"].shape[0]
    t, tp = _theta(theta)
    g = np.zeros(mpnn_nparams()) if grad else None
    er = np.ascontiguousarray(er, dtype=np.float64)
    b = _f64(b, (n, 3))
    xstar = _f64(xstar, (n, 3))
    if norm not in ("A", "2"):
        raise ValueError("norm must be 'A' or '2'")
    loss = lib().orc_mpnn_loss_grad_norm(n, _ip(sys_["rowptr"]), _ip(sys_["col"]),
                                         _dp(sys_["val"]), _dp(sys_["diag"]), _dp(er),
                                         float(alpha), tp, _dp(b), _dp(xstar),
                                         1 if norm == "2" else 0, _dp(g))
    return (loss, g) if grad else loss


def mpnn_block_nparams():
    return int(lib().orc_mpnn_block_nparams())


def _theta_block(theta):
    t = np.ascontiguousarray(theta, dtype=np.float32)
    assert t.shape == (mpnn_block_nparams(),)
    return t, t.ctypes.data_as(C.POINTER(C.c_float))


def mpnn_block_forward(bsys, er, alpha, theta):
    """M^-1 of the learned preconditioner on a block system (build_block_system):
    (mdiag (n, 3, 3), moff (nnz, 3, 3)) in A's block pattern."""
    n = len(bsys["bdiag"])
    t, tp = _theta_block(theta)
    nnz = len(bsys["col"])
    mdiag = np.zeros((n, 3, 3))
    moff = np.zeros((max(nnz, 1), 3, 3))
    er = np.ascontiguousarray(er, dtype=np.float64)
    rc = lib().orc_mpnn_block_forward(n, _ip(bsys["rowptr"]), _ip(np.ascontiguousarray(bsys["col"])),
                                      _dp(np.ascontiguousarray(bsys["bval"])),
                                      _dp(np.ascontiguousarray(bsys["bdiag"])), _dp(er),
                                      float(alpha), tp, _dp(mdiag), _dp(moff))
    if rc != 0:
        raise RuntimeError("oracle block mpnn forward failed")
    return mdiag, moff[:nnz]


def mpnn_block_loss_grad(bsys, er, alpha, theta, b, xstar, grad=True, norm="2"):
    """Loss ||M^-1 b - x*||^2 / ||x*||^2 on a block system in the Euclidean
    (norm "2") or the A-norm and its gradient (mpnn_block_nparams() values)."""
    n = len(bsys["bdiag"])
    t, tp = _theta_block(theta)
    g = np.zeros(mpnn_block_nparams()) if grad else None
    er = np.ascontiguousarray(er, dtype=np.float64)
    b = _f64(b, (n, 3))
    xstar = _f64(xstar, (n, 3))
    if norm not in ("A", "2"):
        raise ValueError("norm must be 'A' or '2'")
    loss = lib().orc_mpnn_block_loss_grad(n, _ip(bsys["rowptr"]),
                                          _ip(np.ascontiguousarray(bsys["col"])),
                                          _dp(np.ascontiguousarray(bsys["bval"])),
                                          _dp(np.ascontiguousarray(bsys["bdiag"])), _dp(er),
                                          float(alpha), tp, _dp(b), _dp(xstar),
                                          1 if norm == "2" else 0, _dp(g))
    return (loss, g) if grad else loss
