"""Exact parity of the decisions stored with the state -- the bin of every particle
in every binning of the observables (section 2) and its cell of the moving prior
(section 2.1) -- against the oracle's FP64 decisions for the same particles,
read through m2m_tags.

The FP32 kernels decide in FP32 outside a guard band around each edge and in FP64
inside it, so every decision must equal the FP64 one exactly (index work:
bit-exact).  The oracle decides from the GPU's own FP32 state, converted to FP64.
"""
import numpy as np
import pytest

import oracle
from synth import configs
from tests import helpers as H
from tests.golden import derive_eps

pytestmark = pytest.mark.gpu

m2m = pytest.importorskip("paper_1207_6403_amd")


def check_tags(cfg, ctx, inp, er, cells=True):
    xv = m2m.m2m_particles(ctx).astype(np.float64)
    t = m2m.m2m_tags(ctx)
    N = xv.shape[1]
    ref = oracle.bins(cfg["layout"], xv[:3])
    nb = ref.shape[0]
    assert t.shape == (nb + 1, N)
    for b in range(nb):
        want = np.where(ref[b] < 0, 0xFFFF, ref[b]).astype(np.uint16)
        bad = np.flatnonzero(t[b] != want)
        H.flush("binning %d (%s): %d particles inside, %d decisions differ" % (
            b, cfg["layout"]["binnings"][b]["kind"], int(np.sum(ref[b] >= 0)), bad.size))
        assert bad.size == 0, (b, bad[:5], t[b][bad[:5]], want[bad[:5]])
    if cells:
        om = oracle.Model(cfg, xv, np.ones(N), inp["Y"], inp["sigma"], Erange=tuple(er))
        want = om.cells()
        bad = np.flatnonzero(t[nb].astype(np.int64) != want)
        H.flush("prior cells: %d distinct, %d decisions differ" % (np.unique(want).size, bad.size))
        assert bad.size == 0, (bad[:5], t[nb][bad[:5]], want[bad[:5]])


def test_tags_headline_full_size():
    """2^20 FP32 particles in the log potential, 64x64 + 20x20 grids, 32x32
    (E, Lz/Lc) cells: the prologue's decisions, then those after three steps."""
    cfg = configs.cfg2()
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case cfg2 N=%d" % cfg["N"])
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    check_tags(cfg, ctx, inp, er)
    m2m.m2m_step(ctx, 3)
    check_tags(cfg, ctx, inp, er)


def test_tags_with_the_derived_energy_range():
    """No energy range given: the library takes min and max of E(0) over the
    particles in FP64, as the oracle's energy_range does."""
    cfg = configs.cfg2(N=1 << 18)
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case cfg2 N=%d, derived energy range" % cfg["N"])
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    check_tags(cfg, ctx, inp, er)
    m2m.m2m_step(ctx, 2)
    check_tags(cfg, ctx, inp, er)


def test_tags_with_a_given_energy_range():
    """A caller's energy range other than the particles' own (wider by a third of
    the span, off-centre) is the one the cells use."""
    cfg = configs.cfg2(N=1 << 16)
    inp = H.inputs(cfg)
    lo, hi = H.erange(cfg, inp)
    er = np.array([lo - 0.25 * (hi - lo), hi + 0.1 * (hi - lo)])
    H.flush("case cfg2 N=%d, energy range %s" % (cfg["N"], er))
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    check_tags(cfg, ctx, inp, er)


def test_tags_multipole_shells():
    """A self-consistent multipole model: sky grids plus 50 spherical shells, cells
    in the analytic reference potential."""
    cfg = configs.cfg3(N=1 << 16, target_n=1 << 16)
    cfg["eps"] = 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case cfg3 N=%d" % cfg["N"])
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    m2m.m2m_step(ctx, 2)
    check_tags(cfg, ctx, inp, er)


def test_tags_separate_cell_kernel():
    """The learned prior's 32x32x8 judge grid, whose cells the separate cell
    kernel decides (period 2: the cells of the state after two steps)."""
    cfg = configs.cfg5(N=30011, target_n=1 << 16)
    cfg["prior"].update(subset=2048, batch=256, period=2)
    cfg["eps"] = 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case cfg5 N=%d" % cfg["N"])
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    m2m.m2m_step(ctx, 2)
    check_tags(cfg, ctx, inp, er)


@pytest.mark.parametrize("pot", ["hernquist", "hernquist_nfw"])
def test_tags_fp32_spherical_potentials(pot):
    """FP32 shells and annuli with an (E, L/Lc) prior in a Hernquist or
    Hernquist + NFW potential: Lc(E) from the closed form or the table."""
    cfg = configs.cfg1(N=1 << 18)
    cfg["precision"] = "f32"
    if pot == "hernquist_nfw":
        cfg["potential"] = {"kind": "hernquist_nfw", "G": 1.0, "M": 1.0, "a": 1.0, "Mh": 5.0, "rs": 4.0}
    # the rate of this model, derived as for the full-size workloads
    cfg["eps"] = 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case cfg1 FP32 %s N=%d" % (pot, cfg["N"]))
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    check_tags(cfg, ctx, inp, er)
    m2m.m2m_step(ctx, 3)
    check_tags(cfg, ctx, inp, er)


def test_tags_fp64_shells_and_annuli():
    cfg = configs.cfg1(N=20000)
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case cfg1 N=%d" % cfg["N"])
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    m2m.m2m_step(ctx, 5)
    check_tags(cfg, ctx, inp, er, cells=cfg["prior"]["kind"] != "flat")
