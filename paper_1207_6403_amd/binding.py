"""ctypes binding of the C ABI in include/m2m.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of the method: it packs Python/numpy/torch arguments into the C
structs, calls the library and unpacks the results.  The library must have been
built (``python -m paper_1207_6403_amd.build``); there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libm2m_hip.so")

ABI_VERSION = 2
MAX_BINNINGS = 4
MLP_NPARAM = 4481
F32, F64 = 0, 1
POT = {"hernquist": 0, "log": 1, "hernquist_nfw": 2, "multipole": 3}
BIN = {"shell": 1, "annulus": 2, "grid": 3}
PRIOR = {"flat": 0, "hist": 1, "mlp": 2}
UPDATE = {"euler": 0, "exp": 1}
STATUS = {0: "OK", 1: "ERR_INVALID", 2: "ERR_NOMEM", 3: "ERR_DEVICE", 4: "ERR_NONPOSITIVE_WEIGHT",
          5: "ERR_NONFINITE", 6: "ERR_UNSUPPORTED"}


class M2MError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class m2m_potential(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lmax", C.c_int32), ("nnode", C.c_int32), ("reserved", C.c_int32),
                ("G", C.c_double), ("M", C.c_double), ("a", C.c_double), ("v0", C.c_double), ("Rc", C.c_double),
                ("q", C.c_double), ("Mh", C.c_double), ("rs", C.c_double), ("rmin", C.c_double),
                ("rmax", C.c_double), ("Mtot", C.c_double)]


class m2m_binning(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nmom", C.c_int32), ("mom", C.c_int32 * 3), ("nedge", C.c_int32),
                ("edges", C.POINTER(C.c_double)), ("nx", C.c_int32), ("ny", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("gh", C.POINTER(C.c_double))]


class m2m_tracers(C.Structure):
    _fields_ = [("binning", C.c_int32), ("n", C.c_int32), ("bin", C.POINTER(C.c_int32)),
                ("v", C.POINTER(C.c_double)), ("width", C.POINTER(C.c_double)), ("lam", C.c_double)]


class m2m_obs_layout(C.Structure):
    _fields_ = [("incl", C.c_double), ("nbin", C.c_int32), ("reserved", C.c_int32),
                ("bin", m2m_binning * MAX_BINNINGS)]


class m2m_prior(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ax2", C.c_int32), ("n", C.c_int32 * 3), ("period", C.c_int32),
                ("Erange", C.POINTER(C.c_double)), ("flat_value", C.c_double), ("ref", m2m_potential),
                ("mlp_subset", C.c_int32), ("mlp_batch", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("adam_eps", C.c_double), ("fallback", C.c_double), ("seed", C.c_uint32),
                ("mlp_mfma", C.c_int32), ("mlp_init", C.POINTER(C.c_float))]


class m2m_config(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("precision", C.c_int32), ("update", C.c_int32), ("frozen", C.c_int32),
                ("dt", C.c_double), ("eps", C.c_double), ("mu", C.c_double), ("tau", C.c_double),
                ("n_models", C.c_int32), ("reserved", C.c_int32), ("model_offsets", C.POINTER(C.c_int64)),
                ("potentials", C.POINTER(m2m_potential)), ("prior", m2m_prior), ("stream", C.c_void_p)]


class m2m_target(C.Structure):
    _fields_ = [("Y", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)), ("J", C.c_int32),
                ("per_model", C.c_int32)]


class m2m_step_stats(C.Structure):
    _fields_ = [("chi2", C.c_double), ("chi2_inst", C.c_double), ("S", C.c_double), ("F", C.c_double),
                ("sum_w", C.c_double), ("min_w", C.c_double), ("sum_w2", C.c_double), ("n_eff", C.c_double),
                ("step", C.c_int64), ("model", C.c_int32), ("reserved", C.c_int32)]


class m2m_launch(C.Structure):
    _fields_ = [("threads", C.c_int32), ("ilp", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("graph_steps", C.c_int32), ("timing", C.c_int32), ("reserved", C.c_int32)]


STAT_FIELDS = ["chi2", "chi2_inst", "S", "F", "sum_w", "min_w", "sum_w2", "n_eff", "step", "model"]
_lib = None
VP = C.c_void_p
CTX = C.c_void_p


def lib():
    """Load libm2m_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError("%s is missing: build it with `python -m paper_1207_6403_amd.build`" % LIB)
        L = C.CDLL(LIB)
        L.m2m_abi_version.restype = C.c_int32
        L.m2m_create.argtypes = [C.POINTER(m2m_config), C.POINTER(m2m_obs_layout), C.POINTER(m2m_target), VP, VP,
                                 C.c_int32, C.POINTER(CTX)]
        L.m2m_step.argtypes = [CTX, C.c_int64, C.POINTER(m2m_step_stats)]
        L.m2m_step_index.argtypes = [CTX]
        L.m2m_step_index.restype = C.c_int64
        L.m2m_observables.argtypes = [CTX, C.c_int32] + [C.POINTER(C.c_double)] * 4
        L.m2m_weights.argtypes = [CTX, VP, C.c_int32]
        L.m2m_priors.argtypes = [CTX, VP, C.POINTER(C.c_double), C.c_int32]
        L.m2m_particles.argtypes = [CTX, VP, C.c_int32]
        L.m2m_tags.argtypes = [CTX, VP, C.c_int32]
        L.m2m_history.argtypes = [CTX, C.POINTER(m2m_step_stats), C.c_int64, C.POINTER(C.c_int64)]
        L.m2m_multipole_tables.argtypes = [CTX, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.m2m_delta_chi2.argtypes = [CTX, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.m2m_shell_moments.argtypes = [CTX, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double)]
        L.m2m_set_tracers.argtypes = [CTX, C.POINTER(m2m_tracers)]
        L.m2m_tracer_state.argtypes = [CTX] + [C.POINTER(C.c_double)] * 3
        L.m2m_mlp_state.argtypes = [CTX, C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int64)]
        L.m2m_mlp_loss_grad.argtypes = [CTX, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int32,
                                        C.POINTER(C.c_float), C.POINTER(C.c_double)]
        L.m2m_mlp_loss_grad_noalloc.argtypes = [CTX, VP, VP, C.c_int32, VP, VP]
        L.m2m_autotune.argtypes = [CTX, C.c_int32, C.POINTER(m2m_launch)]
        L.m2m_get_launch.argtypes = [CTX, C.POINTER(m2m_launch)]
        L.m2m_set_launch.argtypes = [CTX, C.POINTER(m2m_launch)]
        L.m2m_kernel_time.argtypes = [CTX, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.m2m_destroy.argtypes = [CTX]
        L.m2m_destroy.restype = None
        L.m2m_last_error.argtypes = [CTX]
        L.m2m_last_error.restype = C.c_char_p
        for f in ("m2m_create", "m2m_step", "m2m_observables", "m2m_weights", "m2m_priors", "m2m_particles",
                  "m2m_history", "m2m_multipole_tables", "m2m_delta_chi2", "m2m_shell_moments", "m2m_set_tracers", "m2m_tracer_state", "m2m_mlp_state", "m2m_mlp_loss_grad", "m2m_mlp_loss_grad_noalloc", "m2m_autotune", "m2m_get_launch", "m2m_set_launch", "m2m_kernel_time"):
            getattr(L, f).restype = C.c_int
        if L.m2m_abi_version() != ABI_VERSION:
            raise ImportError("libm2m_hip.so ABI %d, binding expects %d" % (L.m2m_abi_version(), ABI_VERSION))
        _lib = L
    return _lib


def _check(status, ctx):
    if status != 0:
        raise M2MError(status, m2m_last_error(ctx))


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ------------------------------------------------------------- struct packing
def pack_potential(p):
    s = m2m_potential()
    s.kind = POT[p["kind"]] if p else -1
    if not p:
        return s
    s.G = float(p.get("G", 1.0))
    s.M = float(p.get("M", 1.0))
    s.a = float(p.get("a", 1.0))
    for k in ("v0", "Rc", "q", "Mh", "rs", "rmin", "rmax", "Mtot"):
        setattr(s, k, float(p.get(k, 0.0)))
    s.lmax = int(p.get("lmax", 0))
    s.nnode = int(p.get("nodes", 0))
    return s


def pack_layout(lay, keep):
    s = m2m_obs_layout()
    s.incl = float(lay["incl"])
    s.nbin = len(lay["binnings"])
    for b, d in enumerate(lay["binnings"]):
        bb = s.bin[b]
        bb.kind = BIN[d["kind"]]
        bb.nmom = len(d["moments"])
        for k, m in enumerate(d["moments"]):
            bb.mom[k] = int(m)
        if d["kind"] == "grid":
            bb.nx, bb.ny = int(d["nx"]), int(d["ny"])
            bb.x0, bb.x1, bb.y0, bb.y1 = (float(d[k]) for k in ("x0", "x1", "y0", "y1"))
        else:
            e = np.ascontiguousarray(d["edges"], dtype=np.float64)
            keep.append(e)
            bb.nedge = e.size
            bb.edges = _dp(e)
        if any(int(m) >= 3 for m in d["moments"]):
            g = np.ascontiguousarray(np.asarray(d["gh"], dtype=np.float64).ravel())   # V_b then sigma_b
            keep.append(g)
            bb.gh = _dp(g)
    return s


def pack_prior(pr, n_models, keep, Erange=None, ref=None):
    s = m2m_prior()
    s.kind = PRIOR[pr["kind"]]
    shape = tuple(pr.get("shape", (1, 1)))
    s.n[0], s.n[1] = int(shape[0]), int(shape[1])
    s.n[2] = int(shape[2]) if len(shape) > 2 else 1
    axes = pr.get("axes", ("E", "L/Lc"))
    s.ax2 = 1 if axes[1] == "Lz/Lc" else 0
    s.period = int(pr.get("period", 1))
    s.flat_value = float(pr.get("flat_value", 0.0))
    s.ref = pack_potential(ref)
    if Erange is not None:
        er = np.ascontiguousarray(Erange, dtype=np.float64).reshape(-1)
        assert er.size == 2 * n_models
        keep.append(er)
        s.Erange = _dp(er)
    s.mlp_subset = int(pr.get("subset", 0))
    s.mlp_batch = int(pr.get("batch", 0))
    s.lr = float(pr.get("lr", 0.0))
    s.beta1 = float(pr.get("beta1", 0.0))
    s.beta2 = float(pr.get("beta2", 0.0))
    s.adam_eps = float(pr.get("adam_eps", 0.0))
    s.fallback = float(pr.get("fallback", 0.0))
    s.seed = int(pr.get("seed", 0)) & 0xFFFFFFFF
    s.mlp_mfma = 1 if pr.get("mfma", False) else 0
    if pr.get("mlp_init") is not None:
        th = np.ascontiguousarray(pr["mlp_init"], dtype=np.float32)
        assert th.size == MLP_NPARAM
        keep.append(th)
        s.mlp_init = th.ctypes.data_as(C.POINTER(C.c_float))
    return s


class Context:
    """Handle of one m2m_ctx plus the host copies the call needed to stay alive."""

    def __init__(self, ptr, n, J, n_models, dtype, ncell, nbin):
        self.ptr = ptr
        self.nbin = nbin
        self.N = n
        self.J = J
        self.n_models = n_models
        self.dtype = dtype
        self.ncell = ncell

    def __del__(self):
        try:
            m2m_destroy(self)
        except Exception:
            pass


def _ptr(ctx):
    return ctx.ptr if isinstance(ctx, Context) else ctx


# ------------------------------------------------------------ entry points
def m2m_abi_version():
    return lib().m2m_abi_version()


def m2m_last_error(ctx=None):
    msg = lib().m2m_last_error(_ptr(ctx) if ctx is not None else None)
    return msg.decode() if msg else ""


def m2m_create(cfg, xv, w, Y, sigma, Erange=None, device_ptrs=False, stream=None, per_model_target=False,
               prior_ref=None):
    """cfg: workload dict (see synth.configs); xv: [6, N] positions and velocities;
    w: [N] weights (numpy arrays, or torch tensors on the GPU with device_ptrs=True)."""
    L = lib()
    keep = []
    prec = F64 if cfg["precision"] == "f64" else F32
    dt = np.float64 if prec == F64 else np.float32
    pots = cfg["potential"] if isinstance(cfg["potential"], list) else [cfg["potential"]]
    M = len(pots)
    if "model_sizes" in cfg:
        offs = np.concatenate([[0], np.cumsum(np.asarray(cfg["model_sizes"], dtype=np.int64))]).astype(np.int64)
    else:
        offs = np.array([0, int(cfg["N"])], dtype=np.int64)
    keep.append(offs)
    parr = (m2m_potential * M)(*[pack_potential(p) for p in pots])
    c = m2m_config()
    c.abi_version = ABI_VERSION
    c.precision = prec
    c.update = UPDATE[cfg.get("update", "exp")]
    c.frozen = 1 if cfg.get("frozen", False) else 0
    c.dt, c.eps, c.mu, c.tau = (float(cfg[k]) for k in ("dt", "eps", "mu", "tau"))
    c.n_models = M
    c.model_offsets = offs.ctypes.data_as(C.POINTER(C.c_int64))
    c.potentials = parr
    if prior_ref is None:
        prior_ref = cfg["prior"].get("ref_potential")
    c.prior = pack_prior(cfg["prior"], M, keep, Erange, prior_ref)
    c.stream = stream
    lay = pack_layout(cfg["layout"], keep)
    Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(-1)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64).reshape(-1)
    t = m2m_target()
    t.Y, t.sigma = _dp(Y), _dp(sigma)
    t.J = Y.size // (M if per_model_target else 1)
    t.per_model = 1 if per_model_target else 0
    if device_ptrs:
        xptr, wptr = int(xv.data_ptr()), int(w.data_ptr())
        n = int(w.numel())
    else:
        xh = np.ascontiguousarray(xv, dtype=dt)
        wh = np.ascontiguousarray(w, dtype=dt)
        keep += [xh, wh]
        xptr, wptr = xh.ctypes.data, wh.ctypes.data
        n = wh.size
    out = CTX()
    st = L.m2m_create(C.byref(c), C.byref(lay), C.byref(t), C.c_void_p(xptr), C.c_void_p(wptr),
                      1 if device_ptrs else 0, C.byref(out))
    if st != 0:
        raise M2MError(st, m2m_last_error(None))
    pr = cfg["prior"]
    ncell = 0 if pr["kind"] == "flat" else int(np.prod(pr["shape"]))
    ctx = Context(out, n, t.J, M, dt, ncell, lay.nbin)
    if cfg.get("tracers"):
        m2m_set_tracers(ctx, cfg["tracers"])
    return ctx


def m2m_set_tracers(ctx, tr):
    """Attach discrete tracers {"binning", "bin", "v", "dv", "h", "lambda"}: kernel
    widths sqrt(dv^2 + h^2)."""
    b = np.ascontiguousarray(tr["bin"], dtype=np.int32)
    v = np.ascontiguousarray(tr["v"], dtype=np.float64)
    wd = np.ascontiguousarray(np.sqrt(np.asarray(tr["dv"], dtype=np.float64) ** 2 + float(tr["h"]) ** 2))
    t = m2m_tracers()
    t.binning, t.n, t.lam = int(tr["binning"]), b.size, float(tr["lambda"])
    t.bin = b.ctypes.data_as(C.POINTER(C.c_int32))
    t.v, t.width = _dp(v), _dp(wd)
    _check(lib().m2m_set_tracers(ctx.ptr, C.byref(t)), ctx)
    ctx.n_tracers = b.size


def m2m_tracer_state(ctx, nb):
    """(log-likelihood, smoothed L per tracer, smoothed M per bin of the tracers'
    binning (nb bins)) of the current state."""
    ll = C.c_double()
    L = np.zeros(ctx.n_tracers)
    M = np.zeros(nb)
    _check(lib().m2m_tracer_state(ctx.ptr, C.byref(ll), _dp(L), _dp(M)), ctx)
    return ll.value, L, M


def _stats_dict(s):
    return {f: getattr(s, f) for f in STAT_FIELDS}


def m2m_step(ctx, n_steps):
    """Advance n_steps; returns the statistics of the last step, one dict per model."""
    rows = (m2m_step_stats * ctx.n_models)()
    _check(lib().m2m_step(ctx.ptr, int(n_steps), rows), ctx)
    return [_stats_dict(r) for r in rows]


def m2m_step_index(ctx):
    return int(lib().m2m_step_index(ctx.ptr))


def m2m_observables(ctx, model=0):
    y, ys, d = (np.zeros(ctx.J) for _ in range(3))
    chi2 = C.c_double()
    _check(lib().m2m_observables(ctx.ptr, model, _dp(y), _dp(ys), _dp(d), C.byref(chi2)), ctx)
    return {"y": y, "y_smooth": ys, "delta": d, "chi2": chi2.value}


def m2m_weights(ctx, out=None):
    """Weights; into a device tensor `out` (torch, on the GPU) or a new numpy array."""
    if out is not None:
        _check(lib().m2m_weights(ctx.ptr, C.c_void_p(int(out.data_ptr())), 1), ctx)
        return out
    w = np.zeros(ctx.N, dtype=ctx.dtype)
    _check(lib().m2m_weights(ctx.ptr, C.c_void_p(w.ctypes.data), 0), ctx)
    return w


def m2m_priors(ctx, cells=True):
    what = np.zeros(ctx.N, dtype=ctx.dtype)
    cm = np.zeros(max(ctx.ncell, 1) * ctx.n_models)
    _check(lib().m2m_priors(ctx.ptr, C.c_void_p(what.ctypes.data), _dp(cm) if (cells and ctx.ncell) else None, 0), ctx)
    return what, (cm.reshape(ctx.n_models, -1) if ctx.ncell else None)


def m2m_particles(ctx, out=None):
    if out is not None:
        _check(lib().m2m_particles(ctx.ptr, C.c_void_p(int(out.data_ptr())), 1), ctx)
        return out
    xv = np.zeros((6, ctx.N), dtype=ctx.dtype)
    _check(lib().m2m_particles(ctx.ptr, C.c_void_p(xv.ctypes.data), 0), ctx)
    return xv


def m2m_tags(ctx, out=None):
    """Stored bin (rows 0..nbin-1, 0xFFFF outside) and prior-cell (row nbin)
    decisions of the current state, [nbin + 1, N] uint16."""
    if out is not None:
        _check(lib().m2m_tags(ctx.ptr, C.c_void_p(int(out.data_ptr())), 1), ctx)
        return out
    t = np.zeros((ctx.nbin + 1, ctx.N), dtype=np.uint16)
    _check(lib().m2m_tags(ctx.ptr, C.c_void_p(t.ctypes.data), 0), ctx)
    return t


def m2m_history(ctx, max_rows=None):
    max_rows = max_rows or 4096 * ctx.n_models
    rows = (m2m_step_stats * max_rows)()
    n = C.c_int64()
    _check(lib().m2m_history(ctx.ptr, rows, max_rows, C.byref(n)), ctx)
    return [_stats_dict(rows[k]) for k in range(n.value)]


def m2m_delta_chi2(ctx):
    """Per-model chi^2 of the last step, chi^2 - min, and the best model's index."""
    chi2 = np.zeros(ctx.n_models)
    delta = np.zeros(ctx.n_models)
    best = C.c_int32()
    _check(lib().m2m_delta_chi2(ctx.ptr, _dp(chi2), _dp(delta), C.byref(best)), ctx)
    return chi2, delta, best.value


def m2m_shell_moments(ctx, edges, model=0):
    """Velocity second moments of a model's weighted particles in spherical shells
    [edges[k], edges[k+1]): array [4, nshell] of sum w, sum w v_r^2,
    sum w v_theta^2, sum w v_phi^2."""
    e = np.ascontiguousarray(edges, dtype=np.float64)
    ns = e.size - 1
    out = np.zeros(4 * max(ns, 0))
    _check(lib().m2m_shell_moments(ctx.ptr, int(model), _dp(e), int(ns), _dp(out)), ctx)
    return out.reshape(4, ns)


def anisotropy(moments):
    """beta = 1 - (sum w v_theta^2 + sum w v_phi^2) / (2 sum w v_r^2) per shell, from
    m2m_shell_moments (second moments about zero: a non-rotating model)."""
    return 1.0 - (moments[2] + moments[3]) / (2.0 * moments[1])


def m2m_multipole_tables(ctx, nnode, lmax):
    """Node coefficient tables (A, B) of a multipole model, each [nnode, (lmax+1)^2]."""
    nlm = (lmax + 1) * (lmax + 1)
    A = np.empty((nnode, nlm))
    B = np.empty((nnode, nlm))
    _check(lib().m2m_multipole_tables(ctx.ptr, _dp(A), _dp(B)), ctx)
    return A, B


def m2m_mlp_state(ctx):
    """Learned prior: parameters (float32 [4481]), last judge value, whether the
    histogram fallback applies, refreshes so far."""
    th = np.empty(MLP_NPARAM, dtype=np.float32)
    j = C.c_double()
    fb = C.c_int32()
    nr = C.c_int64()
    _check(lib().m2m_mlp_state(ctx.ptr, th.ctypes.data_as(C.POINTER(C.c_float)), C.byref(j), C.byref(fb),
                               C.byref(nr)), ctx)
    return {"theta": th, "judge": j.value, "used_fallback": bool(fb.value), "refreshes": nr.value}


def m2m_mlp_loss_grad(ctx, theta, samples):
    """Loss and gradient (float32 [4481]) of the MLP prior's objective over samples
    [n, 4] = (u0, u1, u2, target) at parameters theta, on the GPU."""
    th = np.ascontiguousarray(theta, dtype=np.float32)
    sm = np.ascontiguousarray(samples, dtype=np.float32)
    assert th.size == MLP_NPARAM and sm.ndim == 2 and sm.shape[1] == 4
    g = np.empty(MLP_NPARAM, dtype=np.float32)
    loss = C.c_double()
    fp = C.POINTER(C.c_float)
    _check(lib().m2m_mlp_loss_grad(ctx.ptr, th.ctypes.data_as(fp), sm.ctypes.data_as(fp), sm.shape[0],
                                   g.ctypes.data_as(fp), C.byref(loss)), ctx)
    return loss.value, g


MLP_NOALLOC_MAX = 8192


def m2m_mlp_loss_grad_noalloc(ctx, theta, samples, grad, loss=None):
    """The same loss and gradient with no device allocation: theta (float32 [4481]),
    samples (float32 [n, 4]), grad (float32 [4481]) and loss (float64 [1] or None)
    are device tensors (torch, on the context's device).  Enqueued on the context's
    stream; synchronise before reading grad and loss."""
    n = int(samples.shape[0])
    _check(lib().m2m_mlp_loss_grad_noalloc(ctx.ptr, C.c_void_p(int(theta.data_ptr())),
                                           C.c_void_p(int(samples.data_ptr())), n,
                                           C.c_void_p(int(grad.data_ptr())),
                                           C.c_void_p(int(loss.data_ptr())) if loss is not None else None), ctx)


def _launch_dict(L):
    return {f: getattr(L, f) for f, _ in m2m_launch._fields_ if f != "reserved"}


def m2m_autotune(ctx, trial_steps=10):
    L = m2m_launch()
    _check(lib().m2m_autotune(ctx.ptr, int(trial_steps), C.byref(L)), ctx)
    return _launch_dict(L)


def m2m_get_launch(ctx):
    L = m2m_launch()
    _check(lib().m2m_get_launch(ctx.ptr, C.byref(L)), ctx)
    return _launch_dict(L)


def m2m_set_launch(ctx, **kw):
    L = m2m_launch()
    _check(lib().m2m_get_launch(ctx.ptr, C.byref(L)), ctx)
    for k, v in kw.items():
        setattr(L, k, int(v))
    _check(lib().m2m_set_launch(ctx.ptr, C.byref(L)), ctx)
    return _launch_dict(L)


def m2m_kernel_time(ctx):
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().m2m_kernel_time(ctx.ptr, C.byref(ms), C.byref(n)), ctx)
    return ms.value, n.value


def m2m_destroy(ctx):
    if isinstance(ctx, Context):
        if ctx.ptr:
            lib().m2m_destroy(ctx.ptr)
            ctx.ptr = None
    elif ctx:
        lib().m2m_destroy(ctx)
