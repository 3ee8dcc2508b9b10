"""What the learned warm start gains: on a held-out alloy the FP64 cycle
started from the network's shifts needs fewer iterations to |dq| < 1e-4 than
the same cycle started from zero, and converges to the same energy within
1 meV/atom.  The FP32 -> FP64 precision ladder reaches the same fixed point."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _alloy(seed, reps=6):
    return W.bcc_alloy_scf(seed=seed, reps=reps)


@pytest.fixture(scope="module")
def trained(bop):
    from paper_1803_07491_amd import warmstart as WS
    x, t = WS.training_set([_alloy(6000 + s) for s in range(8)])
    model = WS.fit(x, t, epochs=300, batch=512, lr=3e-3)
    return WS, model


def test_warm_start_gains_iterations(trained):
    WS, model = trained
    test = _alloy(6100)
    plain, it_plain, _, _ = WS.converge(test)
    d0 = WS.predict_shift(model, test)
    rmse = float(((d0 - plain.shift) ** 2).mean().sqrt())
    spread = float(plain.shift.std())
    warm, it_warm, _, _ = WS.converge(test, shift0=d0)
    du = abs(float(warm.out["U_total"].item()) - float(plain.out["U_total"].item())) / test.n_atoms
    print(f"plain {it_plain} iterations, warm {it_warm}; shift rmse {rmse:.2e} (spread {spread:.2e}); dU {du:.2e} eV/atom")
    assert rmse < 0.5 * spread
    assert it_warm < it_plain
    assert du * 1e3 < 1.0


def test_ladder_reaches_fp64_fixed_point(trained):
    WS, model = trained
    test = _alloy(6101)
    plain, it_plain, _, _ = WS.converge(test)
    lad = WS.converge_ladder(test, shift0=WS.predict_shift(model, test))
    du = abs(float(lad.path.out["U_total"].item()) - float(plain.out["U_total"].item())) / test.n_atoms
    print(f"plain {it_plain}; ladder {lad.it_low} FP32 + {lad.it_f64} FP64; dU {du:.2e} eV/atom")
    assert du * 1e3 < 1.0
    assert float(lad.path.max_dq.item()) < 1e-4
    np.testing.assert_allclose(lad.path.shift.cpu().numpy(), plain.shift.cpu().numpy(), atol=2e-3)
