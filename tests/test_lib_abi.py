"""The C-ABI library loads, exports every entry point include/pdt.h declares, and rejects
invalid arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2404_02844_amd import _pdt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pdt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdt_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_symbols()
    assert len(names) >= 9
    L = ctypes.CDLL(_pdt.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def _desc_call(**over):
    base = dict(mu=np.linspace(0, 5, 6), P=np.full((6, 3), 1 / 3), M=8, gamma=0.1, pmf_threshold=1e-16,
                tail_mode=_pdt.PDT_TAIL_LUMP)
    base.update(over)
    return _pdt.pdt_make_problem(base["mu"], base["P"], base["M"], base["gamma"], base["pmf_threshold"],
                                 base["tail_mode"], stream=0)


@pytest.mark.parametrize("over,msg", [
    (dict(mu=np.array([0.0, 2.0, 1.0, 3, 4, 5])), "non-decreasing"),
    (dict(mu=np.array([0.0, -1.0, 1.0, 3, 4, 5])), "mu"),
    (dict(mu=np.array([0.0, np.nan, 1.0, 3, 4, 5])), "mu"),
    (dict(gamma=-1.0), "gamma"),
    (dict(gamma=np.inf), "gamma"),
    (dict(P=np.full((6, 3), np.nan)), "P"),
    (dict(P=-np.ones((6, 3))), "P"),
    (dict(M=0), "M, N and D"),
    (dict(pmf_threshold=1.5), "pmf_threshold"),
    (dict(tail_mode=7), "tail_mode"),
    (dict(P=np.full((6, 300), 1 / 300)), "N must be"),
    (dict(M=200_000_000), "2^31"),
])
def test_invalid_arguments_are_rejected(over, msg):
    with pytest.raises(_pdt.PdtError) as ei:
        _desc_call(**over)
    assert ei.value.status == _pdt.PDT_ERR_INVALID_ARG
    assert msg in str(ei.value)


def test_null_handles_are_rejected():
    L = _pdt.lib()
    opts = _pdt.pdt_solve_opts()
    assert L.pdt_solve(None, None, ctypes.byref(opts), None) == _pdt.PDT_ERR_INVALID_ARG
    f = ctypes.c_double()
    assert L.pdt_objective(None, None, ctypes.byref(f), None) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_project_simplex(None, None, 3, 3, None) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_problem_set_tiles(None, 0, 0, 4, 4) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_problem_tiles(None, 0, 0, None, None) == _pdt.PDT_ERR_INVALID_ARG
    nopts = _pdt.pdt_newton_opts(max_newton=10, cg_max=10)
    assert L.pdt_newton_solve(None, None, ctypes.byref(nopts), None) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_hessian_apply(None, None, None) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_problem_set_fx_split(None, 0, 2) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_problem_fx_split(None, 0, None) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_problem_set_ftr_split(None, 0, 2) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_problem_ftr_split(None, 0, None) == _pdt.PDT_ERR_INVALID_ARG
    assert L.pdt_newton_direction(None, 1, None, 0.0, 1e-4, 10, None, None, None, None) == _pdt.PDT_ERR_INVALID_ARG
    L.pdt_destroy_problem(None)  # no-op
    assert "NULL" in _pdt.pdt_last_error()


def test_model_create_rejects_bad_sizes():
    L = _pdt.lib()
    out = ctypes.c_void_p()
    for sizes in ((0, 8, 8), (258, 0, 16), (258, 8, -1)):
        st = L.pdt_model_create(*sizes, None, None, ctypes.byref(out))
        assert st == _pdt.PDT_ERR_INVALID_ARG and not out.value
    assert "sizes" in _pdt.pdt_last_error()
