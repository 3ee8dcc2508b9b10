"""Learned warm start and precision ladder for the local-charge-neutrality
cycle.

Training data come from the method itself: structures are converged with the
plain FP64 self-consistency (``bop_scf_step`` from zero shifts); each atom
contributes its moment traces mu_1..mu_6 at zero shift (features) and its
converged, gauge-fixed onsite shift (target).  The network is trained with
the library's MLP kernels.  A warm start then costs one cheap 6-moment pass,
the feature kernel and one forward pass; the plain cycle continues from the
predicted shifts and still decides when it has converged.

Precision ladder: with FP32 H.X products the per-atom electron counts carry
noise of order 1e-4..1e-3 electrons at 16 moments (the moments-to-recursion
map amplifies the FP32 rounding of high moments), so an FP32 cycle stalls
above a 1e-4 tolerance.  ``converge_ladder`` therefore runs FP32 steps while
max |q| is well above that floor and hands the shifts to an FP64 cycle, which
finishes and decides convergence: the fixed point and the energies are those
of the FP64 method.

Everything numeric runs in the HIP library; this module only sequences calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

from . import (EnergyPath, MLP, SCFPath, BopError, BOP_E_NOT_CONVERGED, feature_stats, features, mlp_shift,
               standardise, _torch)

N_FEAT_MOMENTS = 6


def zero_shift_features(wl, device="cuda"):
    """Raw features (moment traces 1..6) of the zero-shift Hamiltonian from a
    6-moment pass."""
    p = EnergyPath(wl.pos, wl.cell, wl.species, wl.model, N_FEAT_MOMENTS, wl.n_exp, "f64", device=device)
    p.run_moments()
    return features(p.mu, p.no, N_FEAT_MOMENTS)


def converge(wl, shift0=None, dtype="f64", mix=0.5, tol=1e-4, max_iter=300, device="cuda"):
    """Plain SCF; returns (path, iterations, seconds, history of max|q|).
    The set-up (neighbour list, H, moment plan) is outside the timing."""
    torch = _torch()
    s = SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, dtype, device=device)
    if shift0 is not None:
        s.set_shift(shift0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, hist = s.run_scf(mix=mix, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    return s, it, time.perf_counter() - t0, hist


@dataclass
class LadderResult:
    path: SCFPath            # the FP64 cycle that converged
    it_low: int              # FP32 steps
    it_f64: int              # FP64 steps
    seconds: float
    hist: list


class Ladder:
    """FP32 steps while max|q| >= q_switch, then FP64 steps to ``tol``.
    Both cycles are set up once and can be reused for several starts."""

    def __init__(self, wl, device="cuda"):
        args = (wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp)
        self.low = SCFPath(*args, "f32", device=device)
        self.f64 = SCFPath(*args, "f64", device=device)

    def run(self, shift0=None, q_switch=2e-3, mix=0.5, tol=1e-4, max_low=100, max_iter=300):
        torch = _torch()
        if shift0 is None:
            self.low.shift.zero_()
        else:
            self.low.set_shift(shift0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = []
        it_low = 0
        while it_low < max_low:
            self.low.step(mix, 1e-3, tol)
            it_low += 1
            mq = float(self.low.max_dq.item())
            hist.append(mq)
            if mq < q_switch:
                break
        self.f64.shift.copy_(self.low.shift)
        for it in range(max_iter):
            self.f64.step(mix, 1e-3, tol)
            hist.append(float(self.f64.max_dq.item()))
            if int(self.f64.converged.item()):
                torch.cuda.synchronize()
                return LadderResult(self.f64, it_low, it + 1, time.perf_counter() - t0, hist)
        raise BopError(BOP_E_NOT_CONVERGED, f"SCF not converged in {max_iter} FP64 iterations")


def converge_ladder(wl, shift0=None, **kw):
    return Ladder(wl).run(shift0, **kw)


def training_set(structures, log=None):
    """(features [rows, 6], targets [rows]) device tensors from structures
    converged with the plain FP64 cycle."""
    torch = _torch()
    xs, ts = [], []
    for k, wl in enumerate(structures):
        x = zero_shift_features(wl)
        s, it, sec, _ = converge(wl, dtype="f64")
        xs.append(x)
        ts.append(s.shift.float())
        if log:
            log(f"training structure {k}: {wl.n_atoms} atoms, {it} iterations, {sec:.2f} s")
    return torch.cat(xs), torch.cat(ts)


def fit(x, t, epochs=50, batch=4096, lr=1e-3, seed=0):
    """Standardise the features (``bop_feature_stats``, ``bop_standardise``)
    and train the network; returns the model."""
    m = MLP(seed=seed, device=x.device)
    mean, std = feature_stats(x)
    m.mean.copy_(mean)
    m.std.copy_(std)
    m.train(standardise(x, mean, std), t, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return m


def predict_shift(model, wl):
    """Warm-start shifts for a structure: features of a 6-moment pass,
    standardised with the training statistics, then ``bop_mlp_shift``
    (network output with its mean removed)."""
    p = EnergyPath(wl.pos, wl.cell, wl.species, wl.model, N_FEAT_MOMENTS, wl.n_exp, "f64")
    p.run_moments()
    x = features(p.mu, p.no, N_FEAT_MOMENTS, model.mean, model.std)
    return mlp_shift(model.params, x)
