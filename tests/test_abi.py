"""The C-ABI library loads on a machine without a GPU and exports every
entry point that include/dmrg.h declares (no compute calls); host-only
contexts reject device work with DMRG_ERR_STATE."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dmrg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dmrg_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    import paper_1311_1646_amd as lib
    names = _declared()
    assert {"dmrg_create", "dmrg_build_ops", "dmrg_sigma", "dmrg_renormalize", "dmrg_sweep_ground",
            "dmrg_tda_roots"} <= set(names)
    so = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing


def test_host_only_context_rejects_device_calls():
    import paper_1311_1646_amd as lib
    L = 4
    h = np.eye(L)
    eri = np.zeros((L, L, L, L))
    ctx = lib.Context(L, 2, 2, h, eri, 0.0, device=-1)
    code = lib._lib.dmrg_build_ops(ctx._h, 0)
    assert code == -6  # DMRG_ERR_STATE
    assert b"host-only" in lib._lib.dmrg_last_error(ctx._h) or b"MPS" in lib._lib.dmrg_last_error(ctx._h)
