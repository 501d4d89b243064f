"""Differentiable ground-state energy (torch.autograd) on top of libhubbard.

H is linear in every bond amplitude t_b, on-site repulsion U_i and on-site
energy eps_i (Eq. (count1) with per-bond and per-site parameters), so for a
normalised, non-degenerate ground state psi the Hellmann-Feynman theorem gives
dE0/dtheta = <psi| dH/dtheta |psi>.  The forward pass runs the GPU Lanczos
solve; the backward pass returns the bilinear forms computed by the adjoint
kernel behind ``hub_param_bilinear`` (no autograd through the iteration).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence, Tuple

import numpy as np
import torch

from . import F64, Sector


@dataclass
class _Lattice:
    n_sites: int
    bonds: list
    t: list
    U: list
    eps: list
    n_up: int
    n_dn: int


def _canonical_index(sec: Sector, bonds: Sequence[Tuple[int, int]]) -> np.ndarray:
    bi, bj, _ = sec.bonds()
    where = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(bi, bj))}
    return np.array([where[(min(i, j), max(i, j))] for i, j in bonds], dtype=np.int64)


class GroundEnergy(torch.autograd.Function):
    """E0(t, U, eps) for a fixed lattice (bond list) and sector (N_up, N_dn).

    Inputs are CPU float64 tensors: t per listed bond, U and eps per site.
    Repeated bonds share the gradient of their merged amplitude."""

    @staticmethod
    def forward(ctx, t, U, eps, n_sites, bonds, n_up, n_dn, solver_kw):
        lat = _Lattice(int(n_sites), list(bonds), t.detach().cpu().double().tolist(),
                       U.detach().cpu().double().tolist(), eps.detach().cpu().double().tolist(),
                       int(n_up), int(n_dn))
        sec = Sector(lat)
        try:
            kw = dict(dtype=F64, want_vector=True, tol=1e-13)
            kw.update(solver_kw or {})
            gs = sec.ground_state(**kw)
            db, dU, de = sec.param_bilinear(gs.psi, gs.psi)
            idx = _canonical_index(sec, lat.bonds)
        finally:
            sec.close()
        ctx.save_for_backward(torch.from_numpy(db[idx].copy()), torch.from_numpy(dU.copy()),
                              torch.from_numpy(de.copy()))
        return torch.tensor(gs.e0, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        db, dU, de = ctx.saved_tensors
        return g * db, g * dU, g * de, None, None, None, None, None


def ground_energy(t, U, eps, *, n_sites: int, bonds, n_up: int, n_dn: int, **solver_kw):
    """Differentiable lowest eigenvalue of the (N_up, N_dn) sector."""
    return GroundEnergy.apply(t, U, eps, n_sites, tuple(map(tuple, bonds)), n_up, n_dn, solver_kw)
