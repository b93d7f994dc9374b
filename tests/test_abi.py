"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/mlqmc.h declares, reports its defaults, and validates the
coefficient family before touching a device."""

import os
import re

import numpy as np
import pytest

import paper_2103_03407_amd as m
from synth import coeff_family

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mlqmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mlqmc_[a-z_]+)\s*\(", txt)))


def test_header_declarations_match_exports():
    decl = _declared()
    assert decl == sorted(m.EXPORTS)
    lib = m.load()
    for name in decl:
        assert hasattr(lib, name)


def test_symbols_in_dynamic_table():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", m.binding.LIB_PATH],
                         stdout=subprocess.PIPE, text=True, check=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for name in _declared():
        assert name in syms


def test_default_opts():
    o = m.default_opts()
    assert o.prec == m.MLQMC_FP64
    assert o.eig_rtol == 1e-8 and o.lin_rtol == 0.0 and o.lam_rtol == 0.0 and o.rq_lin_rtol == 1e-2
    assert o.max_rq_iter == 12 and o.max_lin_iter == 60 and o.pcg_graph == 1
    assert o.io_on_device == 0 and o.device_mem_cap == 0 and o.eig_atol == 0.0


@pytest.mark.parametrize("bad", ["nonpositive", "k_zero", "nan"])
def test_create_rejects_invalid_family(bad):
    fam = coeff_family(8)
    fam = dict(fam, c=fam["c"].copy(), k1=fam["k1"].copy())
    if bad == "nonpositive":
        fam["a0"] = 0.5 * float(np.sum(fam["c"]))     # a0 - sum|c|/2 = 0
    elif bad == "k_zero":
        fam["k1"][2] = 0
    else:
        fam["c"][1] = float("nan")
    with pytest.raises(m.MlqmcError) as e:
        m.Context(fam)
    assert e.value.code == m.MLQMC_EINVAL
    assert m.mlqmc_last_error()


def test_no_device_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(m.MlqmcError) as e:
        m.Context(coeff_family(8))
    assert e.value.code == m.MLQMC_EDEVICE


def test_missing_library_raises(tmp_path):
    with pytest.raises(RuntimeError):
        m.binding.load(str(tmp_path / "nope.so"))
