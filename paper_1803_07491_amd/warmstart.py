"""Learned warm start of the local-charge-neutrality cycle.

Training data come from the method itself: structures are converged with the
plain self-consistency (``bop_scf_step`` from zero shifts); each atom
contributes its moment traces mu_1..mu_6 at zero shift (features) and its
converged, gauge-fixed onsite shift (target).  The network is trained with
the library's MLP kernels.  A warm start then costs one cheap 6-moment pass,
the feature kernel and one forward pass; the plain cycle continues from the
predicted shifts and remains the judge of convergence.

Everything numeric runs in the HIP library; this module only sequences calls.
"""
from __future__ import annotations

import time

import numpy as np

from . import EnergyPath, MLP, SCFPath, features, _torch

N_FEAT_MOMENTS = 6


def zero_shift_features(wl, device="cuda"):
    """Raw features (moment traces 1..6) of the zero-shift Hamiltonian from a
    6-moment pass."""
    p = EnergyPath(wl.pos, wl.cell, wl.species, wl.model, N_FEAT_MOMENTS, wl.n_exp, "f64", device=device)
    p.run_moments()
    return features(p.mu, p.no, N_FEAT_MOMENTS)


def converge(wl, shift0=None, dtype="f32", mix=0.5, tol=1e-4, max_iter=300, device="cuda"):
    """Plain SCF; returns (path, iterations, seconds)."""
    torch = _torch()
    s = SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, dtype, device=device)
    if shift0 is not None:
        s.set_shift(shift0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, hist = s.run_scf(mix=mix, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    return s, it, time.perf_counter() - t0, hist


def training_set(structures, dtype="f32", log=None):
    """(features [rows, 6], targets [rows]) device tensors from converged
    structures."""
    torch = _torch()
    xs, ts = [], []
    for k, wl in enumerate(structures):
        x = zero_shift_features(wl)
        s, it, sec, _ = converge(wl, dtype=dtype)
        xs.append(x)
        ts.append(s.shift.float())
        if log:
            log(f"training structure {k}: {wl.n_atoms} atoms, {it} iterations, {sec:.2f} s")
    return torch.cat(xs), torch.cat(ts)


def fit(x, t, epochs=50, batch=4096, lr=1e-3, seed=0):
    """Standardise the features and train the network; returns the model."""
    m = MLP(seed=seed, device=x.device)
    mean = x.mean(0)
    std = x.std(0).clamp_min(1e-12)
    m.mean.copy_(mean)
    m.std.copy_(std)
    m.train((x - mean) / std, t, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return m


def predict_shift(model, wl):
    """Warm-start shifts for a structure (gauge-fixed: mean removed)."""
    p = EnergyPath(wl.pos, wl.cell, wl.species, wl.model, N_FEAT_MOMENTS, wl.n_exp, "f64")
    p.run_moments()
    x = features(p.mu, p.no, N_FEAT_MOMENTS, model.mean, model.std)
    y = model.predict(x).double()
    return y - y.mean()
