"""Plain FP64 propagation of the k-dependent density matrix (paper Section 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings where the paper leaves a choice open:
  * Coupling to A(t): the Peierls substitution k -> k + A/c applied to the
    H0 blocks only (the A-dependent part of Eq. 9 realised as a phase); S(k)
    and the SCC term (Eq. 10) stay at k.  H(k, A) = H0(k + A/c) + H2.
  * Bloch phase: exp(+i (k + A/c) . d) with d = R_J + L - R_I the full bond
    vector (Eqs. 7-8 up to a diagonal unitary gauge, identical observables).
  * Spin-unpolarised occupations f = 2, so Tr(D_k S_k) = N_el per k.
  * Current prefactor (Eq. 14): J = -(1/Omega) sum_k w_k Re Tr(D_k Pi_k)
    with Pi_k = c dH/dA = dH0/dk evaluated at k + A/c.  On the equal-weight
    mesh w_k = 1/N_k this is Eq. 14's -(1/(Omega N_k)) sum_k; with weights the
    current is the k-average the charges and the energy already use.
  * SCC shift of step n is evaluated from the charges of D_n.
  * Leapfrog start (Eq. 13 needs two levels): one forward Euler step.
  * Energy: E = sum_k w_k Re Tr(D_k H0_k(A)) + 1/2 dq^T gamma dq.

The paper's own coupling (Eq. 12) is the second mode, coupling="momentum":
  * H_k(t) = H0_k + (1/c) A . P_k + |A|^2 / (2 c^2) S_k + H2, with the momentum
    matrix P_k^alpha = sum_blocks exp(i k.d) <phi_mu| p^alpha |phi_nu> and
    <phi_mu|p|phi_nu> = i dS/dR_J = i dS(d)/dd (the text after Eq. 12), taken
    from the overlap gradient of each two-centre block; the on-site blocks have
    no gradient (no intra-atomic momentum term in the two-centre form).
  * Current matrix Pi_k = P_k + (A/c) S_k (the text after Eq. 14).
  * Energy: E = sum_k w_k Re Tr(D_k (H0_k + H_ext,k)) + 1/2 dq^T gamma dq.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

C_LIGHT = 137.035999084


def bloch_sum(sysm, values: np.ndarray, kvec: np.ndarray) -> np.ndarray:
    """Dense X_k[mu in I, nu in J] = sum_blocks exp(i k.d) X(I, J, L).

    Eqs. (7)-(8): lattice sum of real-space two-centre blocks with a Bloch
    phase; d is the bond vector of each block.
    """
    no = sysm.norb
    na = sysm.n_atoms
    phase = np.exp(1j * (sysm.blk_d @ kvec))
    m4 = np.zeros((na, na, no, no), dtype=np.complex128)
    np.add.at(m4, (sysm.blk_i, sysm.blk_j), phase[:, None, None] * values)
    return m4.transpose(0, 2, 1, 3).reshape(na * no, na * no)


def overlap_k(sysm, kvec) -> np.ndarray:
    """S_k, Eq. (7).  Independent of the vector potential."""
    return bloch_sum(sysm, sysm.blk_s, np.asarray(kvec, float))


def overlap_inverse(s: np.ndarray) -> np.ndarray:
    """S_k^-1 through a Cholesky factorisation (S_k must be positive definite)."""
    n = s.shape[0]
    c = sla.cho_factor(s, lower=True)
    return sla.cho_solve(c, np.eye(n, dtype=np.complex128))


def h0_k(sysm, kvec, a_vec) -> np.ndarray:
    """H0 part of Eq. (8) with the velocity-gauge shift k -> k + A/c."""
    kk = np.asarray(kvec, float) + np.asarray(a_vec, float) / C_LIGHT
    return bloch_sum(sysm, sysm.blk_h0, kk)


def momentum_k(sysm, kvec, a_vec) -> np.ndarray:
    """Pi_k^alpha = c dH/dA^alpha = dH0/dk^alpha at k + A/c (Eq. 14's current matrix).

    Returns shape (3, N, N): sum over blocks of i d^alpha exp(i(k+A/c).d) H0.
    """
    kk = np.asarray(kvec, float) + np.asarray(a_vec, float) / C_LIGHT
    out = []
    for alpha in range(3):
        vals = 1j * sysm.blk_d[:, alpha][:, None, None] * sysm.blk_h0
        out.append(bloch_sum(sysm, vals, kk))
    return np.stack(out)


def overlap_momentum_k(sysm, kvec) -> np.ndarray:
    """P_k^alpha, shape (3, N, N): Bloch sum of <phi_mu|p^alpha|phi_nu> = i dS/dd^alpha
    over the blocks (Eq. 12 and the text after it)."""
    if sysm.blk_ds is None:
        raise ValueError("the momentum-matrix coupling needs the overlap gradients blk_ds")
    kk = np.asarray(kvec, float)
    return np.stack([bloch_sum(sysm, 1j * sysm.blk_ds[:, alpha], kk) for alpha in range(3)])


def h_ext_k(sysm, kvec, a_vec, s_k) -> np.ndarray:
    """Eq. (12) Bloch-summed: (1/c) A . P_k + |A|^2 / (2 c^2) S_k."""
    a = np.asarray(a_vec, float) / C_LIGHT
    p = overlap_momentum_k(sysm, kvec)
    return np.tensordot(a, p, axes=1) + 0.5 * float(a @ a) * s_k


def field_hamiltonian_k(sysm, kvec, a_vec, s_k, coupling: str = "peierls") -> np.ndarray:
    """The field-dependent one-electron part of H_k(t) (no SCC term)."""
    if coupling == "peierls":
        return h0_k(sysm, kvec, a_vec)
    if coupling == "momentum":
        return h0_k(sysm, kvec, np.zeros(3)) + h_ext_k(sysm, kvec, a_vec, s_k)
    raise ValueError(f"unknown coupling {coupling!r}")


def current_matrix_k(sysm, kvec, a_vec, s_k, coupling: str = "peierls") -> np.ndarray:
    """Pi_k = c dH/dA, shape (3, N, N): dH0/dk at k + A/c (Peierls), or
    P_k + (A/c) S_k (momentum coupling, the text after Eq. 14)."""
    if coupling == "peierls":
        return momentum_k(sysm, kvec, a_vec)
    if coupling == "momentum":
        a = np.asarray(a_vec, float) / C_LIGHT
        return overlap_momentum_k(sysm, kvec) + a[:, None, None] * s_k[None]
    raise ValueError(f"unknown coupling {coupling!r}")


def mulliken(sysm, dens: List[np.ndarray], ovl: List[np.ndarray]) -> np.ndarray:
    """q_I = sum_k w_k Re sum_{mu in I} [D_k S_k]_{mu mu}  (Mulliken population, Section 2)."""
    no = sysm.norb
    q = np.zeros(sysm.n_atoms)
    for w, d, s in zip(sysm.kw, dens, ovl):
        diag = np.real(np.einsum("ij,ji->i", d, s))
        q += w * diag.reshape(sysm.n_atoms, no).sum(axis=1)
    return q


def scc_potential(gamma: np.ndarray, q: np.ndarray, z: np.ndarray) -> np.ndarray:
    """V_I = sum_K gamma_IK dq_K with dq = q - Z (Eq. 10 before the 1/2 (V_I + V_J) split)."""
    return gamma @ (q - z)


def hamiltonian_k(sysm, kvec, a_vec, s_k, v_atom: Optional[np.ndarray],
                  coupling: str = "peierls") -> np.ndarray:
    """H_k(t) = field part + 1/2 (V_I + V_J) S_k^{mu nu}  (Eqs. 8-10, 12): the field
    part is H0(k + A/c) (Peierls) or H0(k) + H_ext (momentum coupling)."""
    h = field_hamiltonian_k(sysm, kvec, a_vec, s_k, coupling)
    if v_atom is not None:
        v_orb = np.repeat(v_atom, sysm.norb)
        h = h + 0.5 * (v_orb[:, None] + v_orb[None, :]) * s_k
    return h


def occupations(eps: np.ndarray, n_electrons: float, tol: float = 1e-8) -> np.ndarray:
    """Aufbau filling with f = 2 per state.

    A degenerate group (spread below tol hartree) that straddles the Fermi
    level shares the electrons left for it equally, so the density stays a
    function of S^-1 H and is therefore stationary and unique.
    """
    n = eps.size
    order = np.argsort(eps, kind="stable")
    e = eps[order]
    f = np.zeros(n)
    left = float(n_electrons)
    i = 0
    while i < n and left > 1e-12:
        j = i + 1
        while j < n and abs(e[j] - e[i]) < tol:
            j += 1
        g = j - i
        take = min(2.0 * g, left)
        f[i:j] = take / g
        left -= take
        i = j
    out = np.zeros(n)
    out[order] = f
    return out


def ground_state(sysm, tol: float = 1e-8):
    """Ground-state density of H0(k) at A = 0 for every k (the starting point of Section 3).

    Solves the generalised problem H0_k C = S_k C eps (C^dag S C = I), fills
    by aufbau, and returns (D0 list, reference charges Z).  Z is the input
    z_ref when given; otherwise the Mulliken charges of D0, which makes D0
    self-consistent (dq = 0 at t = 0) for an SCC run.
    """
    dens, ovl, gaps = [], [], []
    for kvec in sysm.kpts:
        s = overlap_k(sysm, kvec)
        h = h0_k(sysm, kvec, np.zeros(3))
        eps, c = sla.eigh(h, s)
        f = occupations(eps, sysm.n_electrons, tol)
        dens.append((c * f[None, :]) @ c.conj().T)
        ovl.append(s)
        n_occ = int(round(sysm.n_electrons / 2))
        if 0 < n_occ < eps.size:
            es = np.sort(eps)
            gaps.append(es[n_occ] - es[n_occ - 1])
    if sysm.z_ref is not None:
        z = np.asarray(sysm.z_ref, float)
    else:
        z = mulliken(sysm, dens, ovl)
    return dens, z, (min(gaps) if gaps else 0.0)


def density_derivative(s_inv: np.ndarray, h: np.ndarray, d: np.ndarray) -> np.ndarray:
    """dD/dt = -i (S^-1 H D - D H S^-1)  (Eq. 6)."""
    return -1j * (s_inv @ h @ d - d @ h @ s_inv)


def density_derivative_columns(s_inv: np.ndarray, h: np.ndarray, d: np.ndarray, cols) -> np.ndarray:
    """Selected columns of Eq. (6): dD/dt[:, j] = -i (S^-1 (H D[:, j]) - D (H S^-1[:, j])).

    The same expression as density_derivative, evaluated one column at a time
    (O(N^2) per column) so that large systems can be sampled.
    """
    cols = np.asarray(cols)
    return -1j * (s_inv @ (h @ d[:, cols]) - d @ (h @ s_inv[:, cols]))


def observables(sysm, dens, ovl, a_vec, z, coupling: str = "peierls"):
    """Current (Eq. 14), band + SCC energy, Tr(D S) and Mulliken charges of one time level.

    Every k-sum uses the weights w_k; Eq. 14's 1/N_k is the equal-weight case.
    """
    jcur = np.zeros(3)
    e_band = 0.0
    tr = 0.0
    for w, kvec, d, s in zip(sysm.kw, sysm.kpts, dens, ovl):
        pik = current_matrix_k(sysm, kvec, a_vec, s, coupling)
        for alpha in range(3):
            jcur[alpha] += w * np.real(np.trace(d @ pik[alpha]))
        e_band += w * np.real(np.trace(d @ field_hamiltonian_k(sysm, kvec, a_vec, s, coupling)))
        tr += w * np.real(np.trace(d @ s))
    jcur *= -1.0 / sysm.volume
    q = mulliken(sysm, dens, ovl)
    e = e_band
    if sysm.gamma is not None:
        dq = q - z
        e += 0.5 * dq @ sysm.gamma @ dq
    return jcur, e, tr, q


@dataclasses.dataclass
class OracleState:
    d_prev: List[np.ndarray]      # D(t_{n-1}) per k (None before the first step)
    d_cur: List[np.ndarray]       # D(t_n) per k
    step: int
    s: List[np.ndarray]
    s_inv: List[np.ndarray]
    z: np.ndarray


def make_state(sysm, d0, z) -> OracleState:
    """S_k (Eq. 7), S_k^-1 and the first time level, before any step."""
    s = [overlap_k(sysm, k) for k in sysm.kpts]
    s_inv = [overlap_inverse(x) for x in s]
    return OracleState(d_prev=None, d_cur=[np.array(x, dtype=np.complex128) for x in d0],
                       step=0, s=s, s_inv=s_inv, z=np.asarray(z, float))


def propagate(sysm, d0, a_table: np.ndarray, dt: float, n_steps: int, z=None,
              state: Optional[OracleState] = None, coupling: str = "peierls"):
    """Leapfrog integration of Eq. (6) with Eq. (13); records observables.

    Step n (time t_n = n dt) uses A(t_n) = a_table[min(n, len-1)] and the SCC
    potential of the charges of D_n; it records the observables of D_n, then
    forms D_{n+1} = D_{n-1} + 2 dt dD/dt(t_n) (for n = 0: D_1 = D_0 + dt dD/dt).
    Returns (history dict, final OracleState).
    """
    if state is None:
        if z is None:
            z = np.zeros(sysm.n_atoms) if sysm.z_ref is None else sysm.z_ref
        state = make_state(sysm, d0, z)
    hist = {"J": [], "E": [], "trace": [], "q": []}
    a_table = np.asarray(a_table, float).reshape(-1, 3)
    for _ in range(n_steps):
        n = state.step
        a_vec = a_table[min(n, a_table.shape[0] - 1)]
        jcur, e, tr, q = observables(sysm, state.d_cur, state.s, a_vec, state.z, coupling)
        hist["J"].append(jcur)
        hist["E"].append(e)
        hist["trace"].append(tr)
        hist["q"].append(q)
        v = scc_potential(sysm.gamma, q, state.z) if sysm.gamma is not None else None
        new = []
        for ik, kvec in enumerate(sysm.kpts):
            h = hamiltonian_k(sysm, kvec, a_vec, state.s[ik], v, coupling)
            ddot = density_derivative(state.s_inv[ik], h, state.d_cur[ik])
            if state.d_prev is None:
                new.append(state.d_cur[ik] + dt * ddot)
            else:
                new.append(state.d_prev[ik] + 2.0 * dt * ddot)
        state.d_prev, state.d_cur = state.d_cur, new
        state.step += 1
    out = {k: np.asarray(v) for k, v in hist.items()}
    return out, state
