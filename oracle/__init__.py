"""CPU oracle of the NMAGIC made-to-measure per-timestep loop -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is a plain FP64 implementation
(``m2m_oracle.c``, loaded with ctypes, plus ``mlp.py`` in numpy) that shares no
code with the GPU library; both read the same seeded inputs from ``synth``.

Parity pins (tests/test_oracle_*.py) tie it to closed forms, invariants, special
cases and brute force; see the header of ``m2m_oracle.c`` for the step order.
"""
import ctypes as C
import os
import subprocess

import numpy as np

from . import mlp  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "m2m_oracle.c")
LIB = os.path.join(HERE, "_m2m_oracle.so")

MAXBIN = 4
POT_KIND = {"hernquist": 0, "log": 1, "hernquist_nfw": 2, "multipole": 3}
BIN_KIND = {"shell": 1, "annulus": 2, "grid": 3}
PRIOR_KIND = {"flat": 0, "hist": 1, "external": 2, "mlp": 2}
STATUS = {0: "ok", 4: "nonpositive weight", 5: "non-finite weight"}


def build(force=True):
    """Compile the oracle with gcc (strict IEEE, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class Pot(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lmax", C.c_int32), ("nnode", C.c_int32), ("pad", C.c_int32),
                ("G", C.c_double), ("M", C.c_double), ("a", C.c_double), ("v0", C.c_double),
                ("Rc", C.c_double), ("q", C.c_double), ("Mh", C.c_double), ("rs", C.c_double),
                ("rmin", C.c_double), ("rmax", C.c_double), ("Mtot", C.c_double)]


class Layout(C.Structure):
    _fields_ = [("incl", C.c_double), ("nbin", C.c_int32), ("pad", C.c_int32),
                ("kind", C.c_int32 * MAXBIN), ("nmom", C.c_int32 * MAXBIN),
                ("mom", (C.c_int32 * 3) * MAXBIN), ("nedge", C.c_int32 * MAXBIN),
                ("edge", C.POINTER(C.c_double) * MAXBIN),
                ("nx", C.c_int32 * MAXBIN), ("ny", C.c_int32 * MAXBIN),
                ("x0", C.c_double * MAXBIN), ("x1", C.c_double * MAXBIN),
                ("y0", C.c_double * MAXBIN), ("y1", C.c_double * MAXBIN),
                ("gh", C.POINTER(C.c_double) * MAXBIN)]


class Prior(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ax2", C.c_int32), ("n", C.c_int32 * 3), ("period", C.c_int32),
                ("Emin", C.c_double), ("Emax", C.c_double), ("flat_value", C.c_double), ("ref", Pot)]


class Tracers(C.Structure):
    _fields_ = [("binning", C.c_int32), ("n", C.c_int32), ("bin", C.POINTER(C.c_int32)),
                ("v", C.POINTER(C.c_double)), ("s", C.POINTER(C.c_double)), ("lam", C.c_double)]


class Cfg(C.Structure):
    _fields_ = [("N", C.c_int64), ("J", C.c_int32), ("update", C.c_int16), ("frozen", C.c_int16),
                ("dt", C.c_double), ("eps", C.c_double), ("mu", C.c_double), ("tau", C.c_double),
                ("pot", Pot), ("lay", Layout), ("prior", Prior),
                ("Y", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)), ("trc", Tracers)]


class State(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in
                ("x", "y", "z", "vx", "vy", "vz", "w", "what", "ys", "yobs", "delta", "mpA", "mpB")] + \
               [("n", C.c_int64)] + [(n, C.c_double) for n in
                                     ("chi2", "chi2_inst", "S", "F", "sumw", "minw", "sumw2")] + \
               [("status", C.c_int32), ("pad", C.c_int32), ("bad_step", C.c_int64)] + \
               [(n, C.POINTER(C.c_double)) for n in ("tL", "tM", "tLobs", "tMobs")] + [("loglike", C.c_double)]


def tracer_widths(tr):
    """Kernel width of each tracer: sqrt(error^2 + h^2)."""
    return np.sqrt(np.asarray(tr["dv"], dtype=np.float64) ** 2 + float(tr["h"]) ** 2)


def make_tracers(tr, keep):
    """Tracers struct from {"binning", "bin", "v", "dv", "h", "lambda"} (or None)."""
    t = Tracers()
    t.binning, t.n, t.lam = -1, 0, 0.0
    if not tr:
        return t
    b = np.ascontiguousarray(tr["bin"], dtype=np.int32)
    v = _f64(tr["v"])
    sw = tracer_widths(tr)
    keep += [b, v, sw]
    t.binning, t.n, t.lam = int(tr["binning"]), b.size, float(tr["lambda"])
    t.bin = b.ctypes.data_as(C.POINTER(C.c_int32))
    t.v, t.s = _dp(v), _dp(sw)
    return t


_lib = None
DP = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        L.or_potential.argtypes = [C.POINTER(Pot), C.c_double, C.c_double, C.c_double, DP, DP, DP, DP]
        L.or_circular_L.argtypes = [C.POINTER(Pot), C.c_double]
        L.or_circular_L.restype = C.c_double
        L.or_kernel.argtypes = [C.POINTER(Layout)] + [C.c_double] * 6 + [C.POINTER(C.c_int32), DP]
        L.or_kernel.restype = C.c_int
        L.or_cell.argtypes = [C.POINTER(Prior)] + [C.c_double] * 6
        L.or_bins.argtypes = [C.POINTER(Layout), C.c_int64, DP, DP, DP, C.POINTER(C.c_int32)]
        L.or_cells.argtypes = [C.POINTER(Prior), C.c_int64] + [DP] * 6 + [C.POINTER(C.c_int32)]
        L.or_prior_means.argtypes = [C.POINTER(Prior), C.c_int64] + [DP] * 10
        L.or_integrals.argtypes = [C.POINTER(Prior), C.c_int64] + [DP] * 10
        L.or_legendre.argtypes = [C.c_int, C.c_double, DP]
        L.or_mp_coeffs.argtypes = [C.POINTER(Pot), C.c_int64, DP, DP, DP, DP, DP, DP]
        L.or_mp_eval.argtypes = [C.POINTER(Pot), DP, DP, C.c_double, C.c_double, C.c_double, DP, DP, DP, DP]
        L.or_mp_exact.argtypes = [C.POINTER(Pot), C.c_int64, DP, DP, DP, DP,
                                  C.c_double, C.c_double, C.c_double, DP, DP, DP, DP]
        L.or_observe.argtypes = [C.POINTER(Cfg), C.c_int64] + [DP] * 8
        L.or_tracer_observe.argtypes = [C.POINTER(Cfg), C.c_int64] + [DP] * 9
        L.or_leapfrog.argtypes = [C.POINTER(Pot), C.c_int64, C.c_int64, C.c_double] + [DP] * 6
        L.or_field_many.argtypes = [C.POINTER(Pot), DP, DP, C.c_int64] + [DP] * 7
        L.or_step.argtypes = [C.POINTER(Cfg), C.POINTER(State)]
        L.or_run.argtypes = [C.POINTER(Cfg), C.POINTER(State), C.c_int64, DP]
        L.or_philox4x32.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.or_subset.argtypes = [C.c_uint32, C.c_uint32, C.c_int64, C.c_uint32, C.POINTER(C.c_int64)]
        L.or_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(DP)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------- struct builders
def make_pot(p):
    s = Pot()
    s.kind = POT_KIND[p["kind"]]
    for k in ("G", "M", "a", "v0", "Rc", "q", "Mh", "rs", "rmin", "rmax", "Mtot"):
        setattr(s, k, float(p.get(k, 0.0)))
    if p["kind"] in ("hernquist", "hernquist_nfw", "multipole"):
        s.G = float(p.get("G", 1.0))
    if p["kind"] == "hernquist":
        s.M, s.a = float(p.get("M", 1.0)), float(p.get("a", 1.0))
    s.lmax = int(p.get("lmax", 0))
    s.nnode = int(p.get("nodes", 0))
    return s


def make_layout(lay, keep):
    s = Layout()
    s.incl = float(lay["incl"])
    s.nbin = len(lay["binnings"])
    assert s.nbin <= MAXBIN
    for b, d in enumerate(lay["binnings"]):
        s.kind[b] = BIN_KIND[d["kind"]]
        s.nmom[b] = len(d["moments"])
        for m, mo in enumerate(d["moments"]):
            s.mom[b][m] = int(mo)
        if any(int(mo) >= 3 for mo in d["moments"]):
            gh = _f64(np.asarray(d["gh"], dtype=np.float64).ravel())   # V_b then sigma_b
            keep.append(gh)
            s.gh[b] = _dp(gh)
        if d["kind"] in ("shell", "annulus"):
            e = _f64(d["edges"])
            keep.append(e)
            s.nedge[b] = e.size
            s.edge[b] = _dp(e)
        else:
            s.nx[b], s.ny[b] = int(d["nx"]), int(d["ny"])
            s.x0[b], s.x1[b], s.y0[b], s.y1[b] = d["x0"], d["x1"], d["y0"], d["y1"]
    return s


def make_prior(pr, pot, N, Erange):
    s = Prior()
    s.kind = PRIOR_KIND[pr["kind"]]
    axes = pr.get("axes", ("E", "L/Lc"))
    s.ax2 = 1 if axes[1] == "Lz/Lc" else 0
    shape = tuple(pr.get("shape", (1, 1)))
    s.n[0], s.n[1] = shape[0], shape[1]
    s.n[2] = shape[2] if len(shape) > 2 else 1
    s.period = int(pr.get("period", 1))
    s.flat_value = float(pr.get("flat_value", 1.0 / N))
    ref = pr.get("ref_potential", pot if pot["kind"] != "multipole" else None)
    if ref is None:
        from synth.configs import LOG_POT
        ref = LOG_POT
    s.ref = make_pot(ref)
    if Erange is not None:
        s.Emin, s.Emax = float(Erange[0]), float(Erange[1])
    return s


def prior_ref_potential(cfg, model=0):
    pot = cfg["potential"]
    if isinstance(pot, list):
        pot = pot[model]
    ref = cfg["prior"].get("ref_potential")
    if ref is not None:
        return ref
    if pot["kind"] == "multipole":
        from synth.configs import LOG_POT
        return LOG_POT
    return pot


def energies(pot, ics):
    """E = v^2/2 + Phi(x) in an analytic potential (FP64)."""
    L = lib()
    ics = _f64(ics)
    n = ics.shape[1]
    phi, ax, ay, az = (np.empty(n) for _ in range(4))
    P = make_pot(pot)
    x, y, z = (np.ascontiguousarray(ics[k]) for k in range(3))
    L.or_field_many(C.byref(P), None, None, n, _dp(x), _dp(y), _dp(z), _dp(phi), _dp(ax), _dp(ay), _dp(az))
    return 0.5 * (ics[3] ** 2 + ics[4] ** 2 + ics[5] ** 2) + phi


def energy_range(cfg, ics, model_slice=None, model=0):
    """[min E(0), max E(0)] of the initial particles in the prior's potential."""
    pot = prior_ref_potential(cfg, model)
    sub = ics if model_slice is None else ics[:, model_slice]
    E = energies(pot, sub)
    return float(E.min()), float(E.max())


class Model:
    """One M2M model run by the oracle: configuration, owned FP64 state arrays."""

    def __init__(self, cfg, ics, w, Y, sigma, Erange=None, pot=None, model=0):
        L = lib()
        self.cfg = cfg
        self.keep = []
        N = ics.shape[1]
        pot = pot if pot is not None else (cfg["potential"][model] if isinstance(cfg["potential"], list)
                                           else cfg["potential"])
        self.pot = pot
        J = int(sum(len(b["moments"]) * (len(b["edges"]) - 1 if b["kind"] != "grid" else b["nx"] * b["ny"])
                    for b in cfg["layout"]["binnings"]))
        self.J = J
        self.Y = _f64(Y)
        self.sigma = _f64(sigma)
        assert self.Y.size == J and self.sigma.size == J
        c = Cfg()
        c.N, c.J = N, J
        c.dt, c.eps, c.mu, c.tau = cfg["dt"], cfg["eps"], cfg["mu"], cfg["tau"]
        c.update = {"euler": 0, "exp": 1}[cfg.get("update", "exp")]
        c.frozen = 1 if cfg.get("frozen", False) else 0
        c.pot = make_pot(pot)
        c.lay = make_layout(cfg["layout"], self.keep)
        if Erange is None and cfg["prior"]["kind"] != "flat":
            Erange = energy_range({"prior": cfg["prior"], "potential": pot}, ics)
        self.Erange = Erange
        c.prior = make_prior(cfg["prior"], pot, N, Erange)
        c.Y, c.sigma = _dp(self.Y), _dp(self.sigma)
        c.trc = make_tracers(cfg.get("tracers"), self.keep)
        self.c = c
        self.arr = {}
        for k, name in enumerate(("x", "y", "z", "vx", "vy", "vz")):
            self.arr[name] = _f64(ics[k]).copy()
        self.arr["w"] = _f64(w).copy()
        self.arr["what"] = np.full(N, c.prior.flat_value)
        for name in ("ys", "yobs", "delta"):
            self.arr[name] = np.zeros(J)
        nlm = (c.pot.lmax + 1) ** 2
        nn = max(c.pot.nnode, 1)
        self.arr["mpA"] = np.zeros(nn * nlm)
        self.arr["mpB"] = np.zeros(nn * nlm)
        tr = cfg.get("tracers")
        ntb = tracer_bins(cfg["layout"], tr["binning"]) if tr else 1
        self.arr["tL"] = np.zeros(max(c.trc.n, 1))
        self.arr["tLobs"] = np.zeros(max(c.trc.n, 1))
        self.arr["tM"] = np.zeros(ntb)
        self.arr["tMobs"] = np.zeros(ntb)
        s = State()
        for name, a in self.arr.items():
            setattr(s, name, _dp(a))
        s.n = 0
        self.s = s
        if pot["kind"] == "multipole":
            L.or_mp_coeffs(C.byref(c.pot), N, _dp(self.arr["x"]), _dp(self.arr["y"]), _dp(self.arr["z"]),
                           _dp(self.arr["w"]), _dp(self.arr["mpA"]), _dp(self.arr["mpB"]))

    # state views
    def ics(self):
        return np.stack([self.arr[k] for k in ("x", "y", "z", "vx", "vy", "vz")])

    @property
    def w(self):
        return self.arr["w"]

    @property
    def step_index(self):
        return int(self.s.n)

    def run(self, nsteps):
        """Run n steps; returns per-step statistics [n, 8]:
        chi2, chi2_inst, S, F, sum w, min w, sum w^2, step."""
        st = np.zeros((max(nsteps, 1), 8))
        rc = lib().or_run(C.byref(self.c), C.byref(self.s), nsteps, _dp(st))
        self.status = rc
        return st[:nsteps]

    @property
    def loglike(self):
        """Tracer log-likelihood sum_t ln(Ls_t / Ms_b(t)) of the last step's smoothed sums."""
        return float(self.s.loglike)

    def tracer_observe(self):
        """(L_t, M_b) of the current state (no smoothing)."""
        a = self.arr
        L = np.zeros(max(self.c.trc.n, 1))
        M = np.zeros(a["tM"].size)
        lib().or_tracer_observe(C.byref(self.c), self.c.N, _dp(a["x"]), _dp(a["y"]), _dp(a["z"]),
                                _dp(a["vx"]), _dp(a["vy"]), _dp(a["vz"]), _dp(a["w"]), _dp(L), _dp(M))
        return L[:self.c.trc.n], M

    def observe(self):
        y = np.zeros(self.J)
        a = self.arr
        lib().or_observe(C.byref(self.c), self.c.N, _dp(a["x"]), _dp(a["y"]), _dp(a["z"]),
                         _dp(a["vx"]), _dp(a["vy"]), _dp(a["vz"]), _dp(a["w"]), _dp(y))
        return y

    def cells(self):
        a = self.arr
        out = np.zeros(self.c.N, dtype=np.int32)
        lib().or_cells(C.byref(self.c.prior), self.c.N, _dp(a["x"]), _dp(a["y"]), _dp(a["z"]),
                       _dp(a["vx"]), _dp(a["vy"]), _dp(a["vz"]), out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out

    def integrals(self):
        """E, |L|, Lz, Lc(E) of every particle in the prior's reference potential."""
        a = self.arr
        N = self.c.N
        out = [np.empty(N) for _ in range(4)]
        lib().or_integrals(C.byref(self.c.prior), N, _dp(a["x"]), _dp(a["y"]), _dp(a["z"]),
                           _dp(a["vx"]), _dp(a["vy"]), _dp(a["vz"]), *[_dp(o) for o in out])
        return out

    def prior_means(self):
        a = self.arr
        nc = int(np.prod(self.cfg["prior"]["shape"]))
        what = np.zeros(self.c.N)
        cs, cn = np.zeros(nc), np.zeros(nc)
        lib().or_prior_means(C.byref(self.c.prior), self.c.N, _dp(a["x"]), _dp(a["y"]), _dp(a["z"]),
                             _dp(a["vx"]), _dp(a["vy"]), _dp(a["vz"]), _dp(a["w"]), _dp(what), _dp(cs), _dp(cn))
        return what, cs, cn

    def set_what(self, what):
        self.arr["what"][:] = what


def tracer_bins(layout, ib):
    b = layout["binnings"][ib]
    return b["nx"] * b["ny"] if b["kind"] == "grid" else len(b["edges"]) - 1


def kernel_entries(layout, z):
    """Non-zero (j, K_j) of one phase-space point."""
    keep = []
    Lc = make_layout(layout, keep)
    jj = (C.c_int32 * 12)()
    K = (C.c_double * 12)()
    n = lib().or_kernel(C.byref(Lc), *[float(v) for v in z], jj, K)
    return [(jj[e], K[e]) for e in range(n)]


def bins(layout, pos):
    """Bin of every position (pos: [3, N]) in every binning, [nbin, N] int32, -1 outside."""
    keep = []
    Lc = make_layout(layout, keep)
    x, y, z = (_f64(pos[k]) for k in range(3))
    out = np.empty((Lc.nbin, x.size), dtype=np.int32)
    lib().or_bins(C.byref(Lc), x.size, _dp(x), _dp(y), _dp(z), out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out


def circular_L(pot, E):
    P = make_pot(pot)
    return lib().or_circular_L(C.byref(P), float(E))


def potential(pot, x, y, z):
    P = make_pot(pot)
    o = [C.c_double() for _ in range(4)]
    lib().or_potential(C.byref(P), x, y, z, *[C.byref(v) for v in o])
    return tuple(v.value for v in o)


def leapfrog(pot, ics, nsteps, dt):
    P = make_pot(pot)
    a = [_f64(ics[k]).copy() for k in range(6)]
    lib().or_leapfrog(C.byref(P), a[0].size, nsteps, dt, *[_dp(v) for v in a])
    return np.stack(a)


def shell_moments(ics, w, edges):
    """Section 3, Fig. 1: the anisotropy recovered for a spherical target.  Per
    spherical shell [edges[k], edges[k+1]) of r = |x|: sum w, and sum w v_c^2 for
    the spherical velocity components c = r, theta, phi (unit vectors e_r = x/r,
    e_phi = z_hat x e_r / |z_hat x e_r|, e_theta = e_phi x e_r; v_phi = 0 and
    v_theta^2 = |v|^2 - v_r^2 on the z axis).  Returns [4, nshell]."""
    ics = np.asarray(ics, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.float64)
    ns = edges.size - 1
    out = np.zeros((4, ns))
    for i in range(ics.shape[1]):
        x = ics[:3, i]
        v = ics[3:, i]
        r = np.linalg.norm(x)
        k = int(np.searchsorted(edges, r, side="right")) - 1
        if k < 0 or k >= ns:
            continue
        er = x / r
        ephi = np.cross([0.0, 0.0, 1.0], er)
        n = np.linalg.norm(ephi)
        vr = v @ er
        if n > 0.0:
            ephi /= n
            vphi = v @ ephi
            vth = v @ np.cross(ephi, er)
            vth2 = vth * vth
        else:
            vphi = 0.0
            vth2 = v @ v - vr * vr
        out[:, k] += w[i] * np.array([1.0, vr * vr, vth2, vphi * vphi])
    return out


def legendre(lmax, x):
    P = np.zeros((lmax + 1) * (lmax + 1))
    lib().or_legendre(lmax, float(x), _dp(P))
    return P.reshape(lmax + 1, lmax + 1)


def mp_coeffs(pot, pos, w):
    P = make_pot(pot)
    nlm = (P.lmax + 1) ** 2
    A = np.zeros(P.nnode * nlm)
    B = np.zeros(P.nnode * nlm)
    x, y, z = (_f64(pos[k]) for k in range(3))
    w = _f64(w)
    lib().or_mp_coeffs(C.byref(P), x.size, _dp(x), _dp(y), _dp(z), _dp(w), _dp(A), _dp(B))
    return A.reshape(P.nnode, nlm), B.reshape(P.nnode, nlm)


def mp_eval(pot, A, B, pts):
    P = make_pot(pot)
    A, B = _f64(A).ravel(), _f64(B).ravel()
    pts = _f64(pts)
    n = pts.shape[1]
    out = [np.zeros(n) for _ in range(4)]
    x, y, z = (np.ascontiguousarray(pts[k]) for k in range(3))
    lib().or_field_many(C.byref(P), _dp(A), _dp(B), n, _dp(x), _dp(y), _dp(z), *[_dp(o) for o in out])
    return out


def mp_exact(pot, pos, w, pt):
    P = make_pot(pot)
    x, y, z = (_f64(pos[k]) for k in range(3))
    w = _f64(w)
    o = [C.c_double() for _ in range(4)]
    lib().or_mp_exact(C.byref(P), x.size, _dp(x), _dp(y), _dp(z), _dp(w), float(pt[0]), float(pt[1]),
                      float(pt[2]), *[C.byref(v) for v in o])
    return tuple(v.value for v in o)


def philox4x32(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32(c, k, o)
    return list(o)


def subset(seed, refresh, count, N):
    idx = np.zeros(count, dtype=np.int64)
    lib().or_subset(seed, refresh, count, N, idx.ctypes.data_as(C.POINTER(C.c_int64)))
    return idx


def threads():
    return lib().or_threads()


def set_threads(n):
    """Threads of the oracle's parallel loops from now on."""
    lib().or_set_threads(int(n))
