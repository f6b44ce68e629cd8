"""Plain FP64 propagation of the coefficient vectors (Eq. 5) by Crank-Nicolson.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper integrates Eq. 6 by leapfrog and states that it also integrates
Eq. 5, i dC_nk/dt = S_k^-1 H_k C_nk, with the unitary Crank-Nicolson scheme
(Section 2, after Eq. 13).  Written for the generalised problem, one step is

    (S_k + i (dt/2) H_k) C(t + dt) = (S_k - i (dt/2) H_k) C(t),

a Cayley transform of the S-self-adjoint S^-1 H: C^dag S C is conserved
exactly, and with it Tr(D_k S_k), for any H.  The density is
D_k = sum_n f_n C_nk C_nk^dag (the definition after Eq. 6) and the charges,
current and energy are those of the density form (Eq. 10, Eq. 14).

Readings where the paper leaves a choice open:
  * H of the step t_n -> t_{n+1} is taken at the midpoint: the field
    A_{n+1/2} = (A(t_n) + A(t_{n+1}))/2 from the A(t_n) table (past its end the
    last entry), and the SCC potential extrapolated from the last two charge
    sets, V_{n+1/2} = (3 V_n - V_{n-1})/2 (V_{-1} = V_0 on the first step).
    Both keep the scheme second order for a time-dependent, self-consistent H
    while each step needs a single linear solve.
  * Step n records the observables of C_n with A(t_n), as the density form does.
  * Occupations are those of the aufbau ground state (f = 2, a degenerate
    group at the Fermi level sharing its electrons), fixed for the run.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .tddftb import (hamiltonian_k, h0_k, mulliken, observables, occupations, overlap_k,
                     scc_potential)


def density_from_coefficients(c: np.ndarray, f: np.ndarray) -> np.ndarray:
    """D_k = sum_n f_n C_n C_n^dag for the columns C_n of c (the definition after Eq. 6)."""
    return (c * f[None, :]) @ c.conj().T


def ground_state_coefficients(sysm, tol: float = 1e-8):
    """Occupied generalised eigenvectors of H0_k C = S_k C eps at A = 0.

    Returns (coefficient list of N x n_s arrays, occupations n_k x n_s,
    reference charges Z, smallest HOMO-LUMO gap).  n_s is the largest number of
    states with f > 0 over k; columns are in ascending eigenvalue order, and a
    k-point with fewer occupied states carries its next states with f = 0.
    C^dag S C = I.  Z is z_ref when given, else the Mulliken charges of the
    ground state.
    """
    vecs, occs, ovl, gaps = [], [], [], []
    for kvec in sysm.kpts:
        s = overlap_k(sysm, kvec)
        h = h0_k(sysm, kvec, np.zeros(3))
        eps, c = sla.eigh(h, s)
        vecs.append(c)
        occs.append(occupations(eps, sysm.n_electrons, tol))
        ovl.append(s)
        n_occ = int(round(sysm.n_electrons / 2))
        if 0 < n_occ < eps.size:
            gaps.append(eps[n_occ] - eps[n_occ - 1])
    n_s = max(int(np.count_nonzero(f > 0)) for f in occs)
    coeffs = [c[:, :n_s].copy() for c in vecs]
    occ = np.array([f[:n_s] for f in occs])
    if sysm.z_ref is not None:
        z = np.asarray(sysm.z_ref, float)
    else:
        z = mulliken(sysm, [density_from_coefficients(c, f) for c, f in zip(coeffs, occ)], ovl)
    return coeffs, occ, z, (min(gaps) if gaps else 0.0)


@dataclasses.dataclass
class CoefficientState:
    c: List[np.ndarray]            # C(t_n) per k, N x n_s
    occ: np.ndarray                # n_k x n_s occupations
    step: int
    s: List[np.ndarray]
    z: np.ndarray
    v_prev: Optional[np.ndarray]   # SCC potential of the previous step (None at the start)


def make_coefficient_state(sysm, c0, occ, z) -> CoefficientState:
    s = [overlap_k(sysm, k) for k in sysm.kpts]
    return CoefficientState(c=[np.array(x, dtype=np.complex128) for x in c0],
                            occ=np.asarray(occ, float).reshape(sysm.n_k, -1), step=0, s=s,
                            z=np.asarray(z, float), v_prev=None)


def crank_nicolson_step(s: np.ndarray, h: np.ndarray, c: np.ndarray, dt: float) -> np.ndarray:
    """Solve (S + i dt/2 H) C' = (S - i dt/2 H) C for C'."""
    tau = 0.5 * dt
    return np.linalg.solve(s + 1j * tau * h, (s - 1j * tau * h) @ c)


def propagate_crank_nicolson(sysm, c0, occ, a_table: np.ndarray, dt: float, n_steps: int,
                             z=None, state: Optional[CoefficientState] = None,
                             coupling: str = "peierls"):
    """Crank-Nicolson integration of Eq. 5; records the observables of every step.

    Step n (t_n = n dt): observables of D_n = sum f C_n C_n^dag with A(t_n);
    V_n from the charges of D_n; H_k at the midpoint field and the extrapolated
    V_{n+1/2}; one Crank-Nicolson solve per k.  Returns (history, final state).
    """
    if state is None:
        if z is None:
            z = np.zeros(sysm.n_atoms) if sysm.z_ref is None else sysm.z_ref
        state = make_coefficient_state(sysm, c0, occ, z)
    hist = {"J": [], "E": [], "trace": [], "q": []}
    a_table = np.asarray(a_table, float).reshape(-1, 3)
    last = a_table.shape[0] - 1
    for _ in range(n_steps):
        n = state.step
        a_now = a_table[min(n, last)]
        a_mid = 0.5 * (a_table[min(n, last)] + a_table[min(n + 1, last)])
        dens = [density_from_coefficients(c, f) for c, f in zip(state.c, state.occ)]
        jcur, e, tr, q = observables(sysm, dens, state.s, a_now, state.z, coupling)
        hist["J"].append(jcur)
        hist["E"].append(e)
        hist["trace"].append(tr)
        hist["q"].append(q)
        v_mid = None
        if sysm.gamma is not None:
            v_now = scc_potential(sysm.gamma, q, state.z)
            v_mid = v_now if state.v_prev is None else 1.5 * v_now - 0.5 * state.v_prev
            state.v_prev = v_now
        new = []
        for ik, kvec in enumerate(sysm.kpts):
            h = hamiltonian_k(sysm, kvec, a_mid, state.s[ik], v_mid, coupling)
            new.append(crank_nicolson_step(state.s[ik], h, state.c[ik], dt))
        state.c = new
        state.step += 1
    out = {k: np.asarray(v) for k, v in hist.items()}
    return out, state
