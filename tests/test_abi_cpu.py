"""CPU-side checks of the C-ABI library: it loads, exports every declared symbol, and the
pure-host entry points behave as documented (no GPU work is launched here)."""
import ctypes
import os
import re

import pytest

from paper_2606_04895_amd import _abi
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "best.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(best_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_declares_the_four_core_calls():
    names = _declared()
    for n in ("best_init", "best_logL_grad", "best_step", "best_adapt"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_export():
    assert set(_abi.EXPORTS) == set(_declared())


def test_nparams_matches_generator_layout():
    lib = _abi.load()
    for d, w, nh in [(6, 128, 2), (6, 512, 4), (12, 1024, 4), (27, 1024, 5), (3, 64, 1)]:
        assert lib.best_mlp_nparams(d, w, nh) == workloads.mlp_nparams(d, w, nh)
    assert lib.best_mlp_nparams(0, 64, 1) == -1


def test_strerror_codes():
    lib = _abi.load()
    assert lib.best_strerror(0) == b"ok"
    assert b"positive definite" in lib.best_strerror(4)
    assert lib.best_strerror(99) == b"unknown error"


def test_null_handles_are_safe():
    lib = _abi.load()
    lib.best_destroy(None)
    lib.best_trainer_destroy(None)
    assert lib.best_init(None, None, None) == _abi.BEST_EINVAL
    assert lib.best_step(None, 0, 1, None, None) == _abi.BEST_EINVAL
    assert lib.best_adapt(None, None, None) == _abi.BEST_EINVAL
    assert lib.best_logL_grad(None, None, 0, None, None, 0) == _abi.BEST_EINVAL


def test_invalid_problem_rejected_before_device_work():
    lib = _abi.load()
    from paper_2606_04895_amd import _problem_struct
    prob = workloads.make_problem("c2")
    bad = dict(prob, width=100)  # not a multiple of 128
    ps, keep = _problem_struct(bad)
    cfg = _abi.Config()
    cfg.n_chains = 16
    h = ctypes.c_void_p()
    assert lib.best_init(ctypes.byref(h), ctypes.byref(ps), ctypes.byref(cfg)) == _abi.BEST_EINVAL
    assert not h.value
