"""CPU-side checks of the C ABI's argument validation: calls with sizes or
options outside what an entry point supports return the documented error
code and a message from bop_last_error, before any device work is enqueued
(these paths make no HIP call, so they run without a GPU).  Workspace-size
queries are host arithmetic and are checked the same way."""
import ctypes as C
import os

import pytest

import paper_1803_07491_amd as P

pytestmark = pytest.mark.skipif(not os.path.exists(P.LIB_PATH), reason="library not built")


def _lib():
    return P.load()


def _err():
    buf = C.create_string_buffer(512)
    _lib().bop_last_error(buf, 512)
    return buf.value.decode()


def _plan(**kw):
    p = P.Plan()
    p.n_atoms, p.n_orb, p.n_max, p.dtype = 128, 5, 9, P.DTYPES["f64"]
    p.n_tiles, p.batch_tiles, p.tile_atoms = 11, 11, 12
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_weights_reject_orders_beyond_twenty():
    lib = _lib()
    assert lib.bop_weights_workspace_size(10, 21) == 0
    assert lib.bop_weights_workspace_size(10, 20) > 0
    rc = lib.bop_weights(4, 21, 200, None, None, None, None, None, 0, None)
    assert rc == P.BOP_E_UNSUPPORTED and "n_max" in _err()
    assert lib.bop_weights(-1, 8, 200, None, None, None, None, None, 0, None) == P.BOP_E_ARG


def test_forces_reject_unsupported_plans_before_any_work():
    lib = _lib()
    for kw, code, word in (({"n_orb": 9}, P.BOP_E_UNSUPPORTED, "d band"),
                           ({"dtype": P.DTYPES["bf16"]}, P.BOP_E_UNSUPPORTED, "FP64 or FP32"),
                           ({"n_max": 21}, P.BOP_E_UNSUPPORTED, "n_max"),
                           ({"r_max": 5.0}, P.BOP_E_UNSUPPORTED, "radius")):
        plan = _plan(**kw)
        rc = lib.bop_forces(C.byref(plan), None, None, None, None, 0, None, None, None, None, 0, None, None, None,
                            0, None)
        assert rc == code, kw
        assert word in _err(), (kw, _err())
    assert lib.bop_forces(None, None, None, None, None, 0, None, None, None, None, 0, None, None, None, 0,
                          None) == P.BOP_E_ARG
    # a supported plan with no atoms does nothing and succeeds
    assert lib.bop_forces(C.byref(_plan(n_atoms=0)), None, None, None, None, 0, None, None, None, None, 0, None,
                          None, None, 0, None) == P.BOP_OK
    assert lib.bop_forces_workspace_size(None, 0, 0) == 0
    assert lib.bop_forces_workspace_size(C.byref(_plan(n_max=25)), 100, 8) == 0


def test_scf_target_and_mlp_update_arguments():
    lib = _lib()
    assert lib.bop_scf_target(-1, 5, None, None, None, None) == P.BOP_E_ARG
    assert lib.bop_scf_target(0, 5, None, None, None, None) == P.BOP_OK
    assert lib.bop_scf_target(3, 5, None, None, None, None) == P.BOP_E_ARG and "NULL" in _err()
    assert lib.bop_mlp_adam(None, None, None, None, 1, 1e-3, None) == P.BOP_E_ARG
    g = C.c_void_p(16)      # never dereferenced: the step is rejected first
    assert lib.bop_mlp_adam(g, g, g, g, 0, 1e-3, None) == P.BOP_E_ARG and "step" in _err()


def test_batched_moments_reject_missing_plan_and_path_radius():
    lib = _lib()
    args = [1, None, None, None, None, None, None, None, None, None, None, None, None, 0, None]
    assert lib.bop_moments_batched(None, *args) == P.BOP_E_ARG
    assert lib.bop_moments_batched(C.byref(_plan(r_max=4.0)), *args) == P.BOP_E_UNSUPPORTED
    assert "radius" in _err()
