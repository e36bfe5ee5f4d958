"""ctypes marshalling for ``libsem.so`` (see include/sem.h for the meaning of every call)."""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libsem.so")

SEM_F64, SEM_F32, SEM_F32_GBF16, SEM_F32_GCOL = 0, 1, 2, 3
SEM_SMOOTH_JACOBI, SEM_SMOOTH_CHEBYSHEV, SEM_SMOOTH_SCHWARZ = 0, 1, 2
SEM_OUTER_FPCG, SEM_OUTER_PDC, SEM_OUTER_GMRES = 0, 1, 2
SEM_FACE_TOP = 1
SEM_MAX_LEVELS = 8

STATUS = {0: "SEM_OK", 1: "SEM_ERR_ARG", 2: "SEM_ERR_ALLOC", 3: "SEM_ERR_HIP",
          4: "SEM_ERR_NOT_CONVERGED", 5: "SEM_ERR_BREAKDOWN", 6: "SEM_ERR_STATE"}


class SemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("ne", ctypes.c_int * 3), ("order", ctypes.c_int),
        ("nlevels", ctypes.c_int), ("level_order", ctypes.c_int * SEM_MAX_LEVELS),
        ("len", ctypes.c_double * 2), ("h", ctypes.POINTER(ctypes.c_double)),
        ("eta", ctypes.POINTER(ctypes.c_double)), ("dirichlet_faces", ctypes.c_uint),
        ("inner_prec", ctypes.c_int), ("smoother", ctypes.c_int), ("nu_pre", ctypes.c_int),
        ("nu_post", ctypes.c_int), ("cheb_degree", ctypes.c_int),
        ("jacobi_omega", ctypes.c_double), ("cheb_lo", ctypes.c_double),
        ("cheb_hi", ctypes.c_double), ("outer", ctypes.c_int), ("maxit", ctypes.c_int),
        ("lanczos_steps", ctypes.c_int), ("lanczos_seed", ctypes.c_ulonglong),
        ("stream", ctypes.c_void_p), ("coarse_dense_max", ctypes.c_int),
        ("gmres_restart", ctypes.c_int), ("order_z", ctypes.c_int),
        ("level_order_z", ctypes.c_int * SEM_MAX_LEVELS), ("precond_still_water", ctypes.c_int),
        ("schwarz_overlap", ctypes.c_int), ("cheb_degree_coarse", ctypes.c_int),
    ]


class JudgeResult(ctypes.Structure):
    _fields_ = [("rho_plain", ctypes.c_double), ("rho_learned", ctypes.c_double),
                ("ms_plain", ctypes.c_double), ("ms_learned", ctypes.c_double),
                ("enabled", ctypes.c_int)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("val_frac", ctypes.c_float), ("seed", ctypes.c_ulonglong),
                ("init", ctypes.c_void_p), ("init_nbytes", ctypes.c_size_t)]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int), ("vcycles", ctypes.c_int), ("learned_skips", ctypes.c_int),
        ("rel_res", ctypes.c_double), ("ms", ctypes.c_double), ("nhist", ctypes.c_int),
        ("hist", ctypes.c_double * 512), ("stage_off_at", ctypes.c_int),
    ]

    def history(self):
        return list(self.hist[: self.nhist])


_lib = None


def lib_path():
    return _LIB_PATH


def lib():
    """Load libsem.so (raises RuntimeError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run python -m paper_2411_14977_amd.build")
    # torch first: its HIP runtime is then the one the library binds to, the runtime that owns
    # the device pointers and streams passed in (loaded alone, the library would bind the
    # system runtime, a second one in the process)
    import torch  # noqa: F401
    L = ctypes.CDLL(_LIB_PATH)
    vp, dp, ip, sz = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "sem_mesh_desc_default": (None, [ctypes.POINTER(MeshDesc)]),
        "sem_mesh_setup": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)]),
        "sem_destroy": (None, [vp]),
        "sem_get_sizes": (ctypes.c_int, [vp, sz, sz, sz]),
        "sem_num_levels": (ctypes.c_int, [vp]),
        "sem_get_level": (ctypes.c_int, [vp, ip, ctypes.POINTER(ctypes.c_int), sz,
                                         ctypes.POINTER(ctypes.c_double)]),
        "sem_get_level_orders": (ctypes.c_int, [vp, ip, ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int)]),
        "sem_gll": (ctypes.c_int, [ip, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]),
        "sem_node_coords": (ctypes.c_int, [vp, ip, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]),
        "sem_apply_laplacian": (ctypes.c_int, [vp, dp, dp]),
        "sem_apply_level": (ctypes.c_int, [vp, ip, dp, dp]),
        "sem_pmg_vcycle": (ctypes.c_int, [vp, dp, dp]),
        "sem_poisson_solve": (ctypes.c_int, [vp, dp, dp, ctypes.c_double,
                                             ctypes.POINTER(SolveInfo)]),
        "sem_assemble_rhs": (ctypes.c_int, [vp, dp, dp, dp, dp]),
        "sem_set_smoother_bounds": (ctypes.c_int, [vp, ip, ctypes.c_double]),
        "sem_restrict": (ctypes.c_int, [vp, ip, dp, dp, dp]),
        "sem_prolong_add": (ctypes.c_int, [vp, ip, dp, dp]),
        "sem_smooth": (ctypes.c_int, [vp, ip, ip, dp, dp]),
        "sem_coarse_solve": (ctypes.c_int, [vp, dp, dp]),
        "sem_time_operator": (ctypes.c_int, [vp, ip, ip, ip, ip, ctypes.POINTER(ctypes.c_double)]),
        "sem_operator_bytes": (ctypes.c_int, [vp, ip, ip, ctypes.POINTER(ctypes.c_double)]),
        "sem_solve_bytes": (ctypes.c_int, [vp, dp, dp, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_long)]),
        "sem_mlp_blob_size": (ctypes.c_size_t, [ip, ip]),
        "sem_learned_features": (ctypes.c_int, [vp, dp, dp, dp, dp]),
        "sem_mlp_train": (ctypes.c_int, [dp, dp, ip, ip, ip, ctypes.POINTER(TrainCfg), vp,
                                         ctypes.c_size_t, ctypes.POINTER(ctypes.c_float)]),
        "sem_mlp_forward": (ctypes.c_int, [vp, ctypes.c_size_t, dp, ip, dp]),
        "sem_learned_harvest": (ctypes.c_int, [vp, dp, ip, ip, ctypes.c_ulonglong, dp, dp,
                                               ctypes.POINTER(ctypes.c_size_t)]),
        "sem_learned_train": (ctypes.c_int, [vp, dp, dp, ip, ctypes.POINTER(TrainCfg), vp,
                                             ctypes.POINTER(ctypes.c_size_t)]),
        "sem_mlp_forward_noalloc": (ctypes.c_int, [vp, ctypes.c_size_t, dp, ip, dp]),
        "sem_mlp_gradients": (ctypes.c_int, [vp, ctypes.c_size_t, dp, dp, ip,
                                             ctypes.POINTER(ctypes.c_float),
                                             ctypes.POINTER(ctypes.c_float)]),
        "sem_learned_load": (ctypes.c_int, [vp, vp, ctypes.c_size_t, ip]),
        "sem_mesh_update_surface": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
        "sem_learned_enable": (ctypes.c_int, [vp, ip]),
        "sem_learned_stage": (ctypes.c_int, [vp, dp, dp, ctypes.POINTER(ctypes.c_int)]),
        "sem_learned_skips": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ip]),
        "sem_learned_judge": (ctypes.c_int, [vp, dp, ip, ctypes.POINTER(JudgeResult)]),
        "sem_launch_shape": (ctypes.c_int, [vp, ip, ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int)]),
        "sem_mesh_mixed_stage": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double)]),
        "sem_lserk_coefficients": (None, [ctypes.POINTER(ctypes.c_double)] * 3),
        "sem_lserk_update": (ctypes.c_int, [vp, ip, ctypes.c_double, dp, dp, dp,
                                            ctypes.c_size_t]),
        "sem_surface_dz": (ctypes.c_int, [vp, dp, dp]),
        "sem_wave_rhs": (ctypes.c_int, [vp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                        ctypes.POINTER(SolveInfo)]),
        "sem_wave_step": (ctypes.c_int, [vp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.POINTER(ctypes.c_int)]),
        "sem_last_error": (ctypes.c_char_p, [vp]),
        "sem_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(ctx, status):
    if status != 0:
        msg = lib().sem_last_error(ctx)
        raise SemError(status, msg.decode() if msg else "")
    return status


def _ptr32(t):
    """Device pointer of a contiguous float32 CUDA tensor."""
    if t is None:
        return None
    if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 4 and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _ptr(t):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


# ---- C ABI mirrors ---------------------------------------------------------------------------
def sem_mesh_desc_default():
    d = MeshDesc()
    lib().sem_mesh_desc_default(ctypes.byref(d))
    return d


def sem_mesh_setup(desc):
    h = ctypes.c_void_p()
    st = lib().sem_mesh_setup(ctypes.byref(desc), ctypes.byref(h))
    if st != 0:
        msg = lib().sem_last_error(None)
        raise SemError(st, msg.decode() if msg else "")
    return h


def sem_destroy(ctx):
    lib().sem_destroy(ctx)


def sem_get_sizes(ctx):
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(ctx, lib().sem_get_sizes(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def sem_num_levels(ctx):
    return lib().sem_num_levels(ctx)


def sem_get_level(ctx, level):
    o, n, lam = ctypes.c_int(), ctypes.c_size_t(), ctypes.c_double()
    _check(ctx, lib().sem_get_level(ctx, level, ctypes.byref(o), ctypes.byref(n), ctypes.byref(lam)))
    return o.value, n.value, lam.value


def sem_get_level_orders(ctx, level):
    """(order along x, order along sigma) of a level."""
    ox, oz = ctypes.c_int(), ctypes.c_int()
    _check(ctx, lib().sem_get_level_orders(ctx, level, ctypes.byref(ox), ctypes.byref(oz)))
    return ox.value, oz.value


def sem_gll(P):
    r = (ctypes.c_double * (P + 1))()
    w = (ctypes.c_double * (P + 1))()
    st = lib().sem_gll(P, r, w)
    if st != 0:
        raise SemError(st, "bad order")
    return np.array(r[:]), np.array(w[:])


def sem_node_coords(ctx, level, dim=2):
    _, n, _ = sem_get_level(ctx, level)
    x = np.zeros(n)
    y = np.zeros(n)
    z = np.zeros(n)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(ctx, lib().sem_node_coords(ctx, level, x.ctypes.data_as(dp),
                                      y.ctypes.data_as(dp) if dim == 3 else None,
                                      z.ctypes.data_as(dp)))
    return (x, z) if dim == 2 else (x, y, z)


def sem_apply_laplacian(ctx, x, y):
    _check(ctx, lib().sem_apply_laplacian(ctx, _ptr(x), _ptr(y)))


def sem_apply_level(ctx, level, x, y):
    _check(ctx, lib().sem_apply_level(ctx, level, _ptr(x), _ptr(y)))


def sem_pmg_vcycle(ctx, r, z):
    _check(ctx, lib().sem_pmg_vcycle(ctx, _ptr(r), _ptr(z)))


def sem_poisson_solve(ctx, rhs, x, tol, info=None, check=True):
    info = SolveInfo() if info is None else info
    st = lib().sem_poisson_solve(ctx, _ptr(rhs), _ptr(x), float(tol), ctypes.byref(info))
    if check:
        _check(ctx, st)
    return st, info


def sem_assemble_rhs(ctx, f, gN, gD, rhs):
    _check(ctx, lib().sem_assemble_rhs(ctx, _ptr(f), _ptr(gN), _ptr(gD), _ptr(rhs)))


def sem_set_smoother_bounds(ctx, level, lam):
    _check(ctx, lib().sem_set_smoother_bounds(ctx, level, float(lam)))


def sem_restrict(ctx, level, b, x, rc):
    _check(ctx, lib().sem_restrict(ctx, level, _ptr(b), _ptr(x), _ptr(rc)))


def sem_prolong_add(ctx, level, ec, xf):
    _check(ctx, lib().sem_prolong_add(ctx, level, _ptr(ec), _ptr(xf)))


def sem_smooth(ctx, level, pre, b, x):
    _check(ctx, lib().sem_smooth(ctx, level, int(pre), _ptr(b), _ptr(x)))


def sem_coarse_solve(ctx, b, x):
    _check(ctx, lib().sem_coarse_solve(ctx, _ptr(b), _ptr(x)))


def sem_time_operator(ctx, level, kind, reps, flush):
    ms = ctypes.c_double()
    _check(ctx, lib().sem_time_operator(ctx, level, kind, reps, flush, ctypes.byref(ms)))
    return ms.value


def sem_operator_bytes(ctx, level, kind):
    b = ctypes.c_double()
    _check(ctx, lib().sem_operator_bytes(ctx, level, kind, ctypes.byref(b)))
    return b.value


def sem_solve_bytes(ctx, rhs, x, tol):
    """(algorithmic bytes of one solve, its iterations, kernels counted); x is overwritten."""
    b, it, n = ctypes.c_double(), ctypes.c_int(), ctypes.c_long()
    _check(ctx, lib().sem_solve_bytes(ctx, _ptr(rhs), _ptr(x), float(tol), ctypes.byref(b),
                                      ctypes.byref(it), ctypes.byref(n)))
    return b.value, it.value, n.value


def sem_mlp_blob_size(nin, nout):
    return int(lib().sem_mlp_blob_size(nin, nout))


def sem_learned_features(ctx, r, e, X, T):
    _check(ctx, lib().sem_learned_features(ctx, _ptr(r), _ptr(e), _ptr32(X), _ptr32(T)))


def _train_cfg(epochs, batch, lr, val_frac, seed, init):
    cfg = TrainCfg(epochs, batch, lr, val_frac, seed, None, 0)
    if init is not None:
        buf = ctypes.create_string_buffer(bytes(init), len(init))
        cfg.init = ctypes.cast(buf, ctypes.c_void_p)
        cfg.init_nbytes = len(init)
        cfg._keep = buf
    return cfg


def sem_learned_harvest(ctx, b, cycles, per, seed, X, T):
    """Training rows of the context's own p-multigrid into device float32 X, T; returns the
    number of rows written."""
    rows = ctypes.c_size_t()
    _check(ctx, lib().sem_learned_harvest(ctx, _ptr(b), int(cycles), int(per), int(seed),
                                          _ptr32(X), _ptr32(T), ctypes.byref(rows)))
    return rows.value


def sem_learned_train(ctx, X, T, epochs=30, batch=1024, lr=1e-3, val_frac=0.1, seed=1234,
                      init=None):
    """Train the context's stage network on device float32 rows X, T; returns the blob."""
    cfg = _train_cfg(epochs, batch, lr, val_frac, seed, init)
    nb = ctypes.c_size_t(sem_mlp_blob_size(X.shape[1], T.shape[1]))
    blob = ctypes.create_string_buffer(nb.value)
    _check(ctx, lib().sem_learned_train(ctx, _ptr32(X), _ptr32(T), X.shape[0], ctypes.byref(cfg),
                                        blob, ctypes.byref(nb)))
    return bytes(blob.raw[:nb.value])


def sem_mlp_train(X, T, nin, nout, epochs=30, batch=1024, lr=1e-3, val_frac=0.1, seed=1234,
                  init=None):
    """Train on device float32 rows X [n x nin], T [n x nout]; returns (blob bytes, losses)."""
    n = X.shape[0]
    cfg = _train_cfg(epochs, batch, lr, val_frac, seed, init)
    nb = sem_mlp_blob_size(nin, nout)
    blob = ctypes.create_string_buffer(nb)
    losses = (ctypes.c_float * (2 * epochs))()
    _check(None, lib().sem_mlp_train(_ptr32(X), _ptr32(T), n, nin, nout, ctypes.byref(cfg), blob,
                                     nb, losses))
    return bytes(blob.raw), np.array(losses[:]).reshape(epochs, 2)


def sem_mlp_forward(blob, X, nout):
    import torch
    Y = torch.zeros(X.shape[0], nout, dtype=torch.float32, device=X.device)
    _check(None, lib().sem_mlp_forward(blob, len(blob), _ptr32(X), X.shape[0], _ptr32(Y)))
    return Y


def sem_mlp_forward_noalloc(blob, X, nout, Y=None):
    """The allocation-free forward: Y [n x nout] into a caller tensor (allocated here if None)."""
    import torch
    if Y is None:
        Y = torch.zeros(X.shape[0], nout, dtype=torch.float32, device=X.device)
    _check(None, lib().sem_mlp_forward_noalloc(blob, len(blob), _ptr32(X), X.shape[0], _ptr32(Y)))
    return Y


def sem_mlp_gradients(blob, X, T, nparams):
    g = np.zeros(nparams, dtype=np.float32)
    loss = ctypes.c_float()
    _check(None, lib().sem_mlp_gradients(blob, len(blob), _ptr32(X), _ptr32(T), X.shape[0],
                                         g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         ctypes.byref(loss)))
    return g, loss.value


def sem_mesh_update_surface(ctx, eta, refresh=False):
    """New free surface (host array in the layout of the set-up's eta)."""
    e = np.ascontiguousarray(np.asarray(eta, dtype=np.float64).ravel())
    _check(ctx, lib().sem_mesh_update_surface(ctx, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             1 if refresh else 0))


def sem_mesh_mixed_stage(ctx, eta_prev):
    """Mixed-stage outer operator with stage k-1's surface eta_prev (host array; None: back to
    the same-stage operator)."""
    if eta_prev is None:
        _check(ctx, lib().sem_mesh_mixed_stage(ctx, None))
        return
    e = np.ascontiguousarray(np.asarray(eta_prev, dtype=np.float64).ravel())
    _check(ctx, lib().sem_mesh_mixed_stage(ctx, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def sem_lserk_coefficients():
    """(alpha, beta, c) of the five-stage fourth-order low-storage scheme, as numpy arrays."""
    a, b, c = ((ctypes.c_double * 5)() for _ in range(3))
    lib().sem_lserk_coefficients(a, b, c)
    return np.array(a[:]), np.array(b[:]), np.array(c[:])


def sem_lserk_update(ctx, stage, dt, F, K, y):
    _check(ctx, lib().sem_lserk_update(ctx, int(stage), float(dt), _ptr(F), _ptr(K), _ptr(y),
                                       y.numel()))


def sem_surface_dz(ctx, phi, w):
    _check(ctx, lib().sem_surface_dz(ctx, _ptr(phi), _ptr(w)))


def sem_wave_rhs(ctx, y, F, phi, g, tol):
    info = SolveInfo()
    _check(ctx, lib().sem_wave_rhs(ctx, _ptr(y), _ptr(F), _ptr(phi), float(g), float(tol),
                                   ctypes.byref(info)))
    return info


def sem_wave_step(ctx, y, K, phi, dt, g, tol):
    it = (ctypes.c_int * 5)()
    _check(ctx, lib().sem_wave_step(ctx, _ptr(y), _ptr(K), _ptr(phi), float(dt), float(g),
                                    float(tol), it))
    return list(it[:])


def sem_learned_load(ctx, blob, enable=True):
    _check(ctx, lib().sem_learned_load(ctx, blob, len(blob), int(enable)))


def sem_learned_enable(ctx, enable):
    _check(ctx, lib().sem_learned_enable(ctx, int(enable)))


def sem_learned_stage(ctx, b, x):
    acc = ctypes.c_int()
    _check(ctx, lib().sem_learned_stage(ctx, _ptr(b), _ptr(x), ctypes.byref(acc)))
    return bool(acc.value)


def sem_learned_judge(ctx, rhs, cycles=6):
    """The plain smoother's verdict on the learned stage (see sem.h): a dict of the per-cycle
    residual reductions and times with the stage off and on, and whether it stays on."""
    r = JudgeResult()
    _check(ctx, lib().sem_learned_judge(ctx, _ptr(rhs), int(cycles), ctypes.byref(r)))
    return {"rho_plain": r.rho_plain, "rho_learned": r.rho_learned, "ms_plain": r.ms_plain,
            "ms_learned": r.ms_learned, "enabled": bool(r.enabled)}


def sem_learned_skips(ctx, reset=False):
    k = ctypes.c_int()
    _check(ctx, lib().sem_learned_skips(ctx, ctypes.byref(k), 1 if reset else 0))
    return k.value


def sem_launch_shape(ctx, level):
    """(fused smoother step columns per workgroup, one-kernel coarse smoothing window)."""
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(ctx, lib().sem_launch_shape(ctx, level, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def blob_pack(nin, nout, W1, b1, W2, b2, W3, b3, seed=0):
    """Network blob (bytes) from FP32 arrays (layout of include/sem.h)."""
    import struct
    hdr = struct.pack("<8IQ2f4I", 0x4E4D4553, 1, nin, 128, nout, 0, 0, 0, seed, 0.0, 0.0, 0, 0, 0, 0)
    body = b"".join(np.ascontiguousarray(a, dtype=np.float32).tobytes() for a in (W1, b1, W2, b2, W3, b3))
    return hdr + body


def blob_unpack(blob):
    import struct
    magic, ver, nin, nh, nout = struct.unpack_from("<5I", blob, 0)
    p = np.frombuffer(blob, dtype=np.float32, offset=64)
    out, off = {}, 0
    for k, shp in (("W1", (nin, nh)), ("b1", (nh,)), ("W2", (nh, nh)), ("b2", (nh,)),
                   ("W3", (nh, nout)), ("b3", (nout,))):
        n = int(np.prod(shp))
        out[k] = p[off:off + n].reshape(shp).astype(np.float64)
        off += n
    return out


# ---- convenience owner of one context -------------------------------------------------------
_PREC = {"f64": SEM_F64, "f32": SEM_F32, "bf16": SEM_F32_GBF16, "col": SEM_F32_GCOL}


class Solver:
    """One solver context.  Inputs h, eta: depth and surface elevation sampled at the fine
    horizontal GLL nodes (use ``fine_x_nodes`` to get them from the library's own rule)."""

    def __init__(self, dim, ne, order, length, h, eta, levels=None, prec="f64",
                 smoother="chebyshev", nu_pre=2, nu_post=2, cheb_degree=3, jacobi_omega=2.0 / 3.0,
                 cheb_lo=0.1, cheb_hi=1.1, outer="fpcg", maxit=500, dirichlet=True,
                 lanczos_steps=20, lanczos_seed=12345, coarse_dense_max=1200, stream=None,
                 gmres_restart=30, order_z=None, precond_still_water=False, schwarz_overlap=0,
                 cheb_degree_coarse=0):
        """order: GLL order (2D: along x); order_z: 2D order along sigma when it differs;
        levels: level orders, each an int or (with order_z) an (x, sigma) pair; None or []:
        the library's own hierarchy."""
        import torch
        d = sem_mesh_desc_default()
        d.dim = dim
        for k in range(3):
            d.ne[k] = int(ne[k])
        d.order = int(order)
        if order_z is not None:
            d.order_z = int(order_z)
        d.precond_still_water = 1 if precond_still_water else 0
        d.schwarz_overlap = int(schwarz_overlap)
        d.cheb_degree_coarse = int(cheb_degree_coarse)
        if levels:
            d.nlevels = len(levels)
            for k, p in enumerate(levels):
                if np.isscalar(p):
                    d.level_order[k] = int(p)
                    d.level_order_z[k] = int(p)
                else:
                    d.level_order[k], d.level_order_z[k] = int(p[0]), int(p[1])
        d.len[0] = float(length[0])
        d.len[1] = float(length[1]) if len(length) > 1 else 1.0
        self._h = np.ascontiguousarray(np.asarray(h, dtype=np.float64).ravel())
        self._eta = np.ascontiguousarray(np.asarray(eta, dtype=np.float64).ravel())
        dp = ctypes.POINTER(ctypes.c_double)
        d.h = self._h.ctypes.data_as(dp)
        d.eta = self._eta.ctypes.data_as(dp)
        d.dirichlet_faces = SEM_FACE_TOP if dirichlet else 0
        d.inner_prec = _PREC[prec]
        d.smoother = {"jacobi": SEM_SMOOTH_JACOBI, "chebyshev": SEM_SMOOTH_CHEBYSHEV,
                      "asm": SEM_SMOOTH_SCHWARZ}[smoother]
        d.nu_pre, d.nu_post, d.cheb_degree = nu_pre, nu_post, cheb_degree
        d.jacobi_omega, d.cheb_lo, d.cheb_hi = jacobi_omega, cheb_lo, cheb_hi
        d.outer = {"fpcg": SEM_OUTER_FPCG, "pdc": SEM_OUTER_PDC, "gmres": SEM_OUTER_GMRES}[outer]
        d.gmres_restart = int(gmres_restart)
        d.maxit = maxit
        d.lanczos_steps = lanczos_steps
        d.lanczos_seed = lanczos_seed
        d.coarse_dense_max = int(coarse_dense_max)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        d.stream = ctypes.c_void_p(int(stream))
        self.dim = dim
        self.ctx = sem_mesh_setup(d)
        self.n_global, self.n_free, self.n_local = sem_get_sizes(self.ctx)
        self.nlevels = sem_num_levels(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            sem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level(self, l):
        return sem_get_level(self.ctx, l)

    def level_orders(self, l):
        return sem_get_level_orders(self.ctx, l)

    def coords(self, level=0):
        return sem_node_coords(self.ctx, level, self.dim)

    def _new(self, n=None):
        import torch
        return torch.zeros(self.n_global if n is None else n, dtype=torch.float64, device="cuda")

    def apply(self, x, y=None):
        y = self._new() if y is None else y
        sem_apply_laplacian(self.ctx, x, y)
        return y

    def apply_level(self, level, x, y=None):
        y = self._new(self.level(level)[1]) if y is None else y
        sem_apply_level(self.ctx, level, x, y)
        return y

    def vcycle(self, r, z=None):
        z = self._new() if z is None else z
        sem_pmg_vcycle(self.ctx, r, z)
        return z

    def solve(self, rhs, x=None, tol=1e-10, check=True):
        x = self._new() if x is None else x
        st, info = sem_poisson_solve(self.ctx, rhs, x, tol, check=check)
        return x, info, st

    def assemble_rhs(self, f=None, gN=None, gD=None):
        rhs = self._new()
        sem_assemble_rhs(self.ctx, f, gN, gD, rhs)
        return rhs

    def set_lambda(self, level, lam):
        sem_set_smoother_bounds(self.ctx, level, lam)

    def update_surface(self, eta, refresh=False):
        sem_mesh_update_surface(self.ctx, eta, refresh)

    def mixed_stage(self, eta_prev):
        sem_mesh_mixed_stage(self.ctx, eta_prev)

    def learned_load(self, blob, enable=True):
        sem_learned_load(self.ctx, blob, enable)

    def learned_enable(self, enable):
        sem_learned_enable(self.ctx, enable)

    def learned_judge(self, rhs, cycles=6):
        return sem_learned_judge(self.ctx, rhs, cycles)

    def smooth(self, level, b, x=None, pre=True):
        x = self._new(self.level(level)[1]) if x is None else x
        sem_smooth(self.ctx, level, pre, b, x)
        return x


def fine_x_nodes(Ne, P, L):
    """Horizontal GLL node coordinates of the fine level from the library's GLL rule."""
    r, _ = sem_gll(P)
    xe = L * (np.arange(Ne)[:, None] + (r[None, :] + 1.0) / 2.0) / Ne
    return np.concatenate([xe[:, :-1].ravel(), [L]])
