"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
entry point declared in include/m2m.h, its structs have the binding's layout, and
invalid arguments are rejected before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "m2m.h")

b = pytest.importorskip("paper_1207_6403_amd.binding")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(m2m_\w+)\s*\(", txt)) - {"m2m_ctx"})


def test_library_exports_every_declared_symbol():
    L = b.lib()
    names = declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", b.LIB], stdout=subprocess.PIPE, text=True).stdout
    exported = set(re.findall(r" T (m2m_\w+)", out))
    assert set(names) <= exported, set(names) - exported


def test_abi_version():
    assert b.m2m_abi_version() == 1


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "m2m.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(m2m_config), '
                   'sizeof(m2m_prior), sizeof(m2m_obs_layout), sizeof(m2m_potential), sizeof(m2m_step_stats), '
                   'sizeof(m2m_launch), sizeof(m2m_target), offsetof(m2m_config, stream), offsetof(m2m_prior, mlp_init));}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(b.m2m_config), C.sizeof(b.m2m_prior), C.sizeof(b.m2m_obs_layout), C.sizeof(b.m2m_potential),
            C.sizeof(b.m2m_step_stats), C.sizeof(b.m2m_launch), C.sizeof(b.m2m_target),
            b.m2m_config.stream.offset, b.m2m_prior.mlp_init.offset]
    assert got == want


def _small():
    cfg = configs.cfg1(N=50)
    inp = configs.make_inputs(cfg)
    return cfg, inp


@pytest.mark.parametrize("mutate,msg", [
    (lambda c, i: c.update(dt=0.0), "dt"),
    (lambda c, i: c.update(mu=-1.0), "mu"),
    (lambda c, i: c.update(tau=0.001), "tau"),
    (lambda c, i: i["w"].__setitem__(3, 0.0), "weights"),
    (lambda c, i: i["w"].__setitem__(3, np.nan), "weights"),
    (lambda c, i: i["ics"].__setitem__((0, 5), np.inf), "coordinate"),
    (lambda c, i: i["sigma"].__setitem__(2, 0.0), "sigma"),
    (lambda c, i: c["layout"]["binnings"][0].__setitem__("edges", np.array([1.0, 0.5, 2.0])), "edges"),
    (lambda c, i: c["prior"].__setitem__("shape", (0, 20)), "prior cells"),
])
def test_invalid_arguments_rejected_without_device(mutate, msg):
    cfg, inp = _small()
    mutate(cfg, inp)
    with pytest.raises(b.M2MError) as e:
        b.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=np.array([-1.0, 0.0]))
    assert e.value.status == 1
    assert msg in str(e.value)


def test_target_size_mismatch_rejected():
    cfg, inp = _small()
    with pytest.raises(b.M2MError) as e:
        b.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"][:-1], inp["sigma"][:-1])
    assert e.value.status == 1
