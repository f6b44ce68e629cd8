"""Pins of the oracle's momentum-matrix coupling (Eq. 12 and the current
matrix after Eq. 14) and of the overlap gradients it reads.

Each check rests on a fact the oracle does not compute itself: finite
differences of the Slater-Koster blocks, the symmetry of the block list,
Hermiticity, time-reversal symmetry of the ground state (so that the
paramagnetic current vanishes and J(0+) of a kick is the closed-form
diamagnetic term), the |A|^2 S term commuting out of Eq. 6 as the paper
notes, the orthogonal-basis limit, energy conservation at constant A, and a
brute-force matrix exponential built here from the raw blocks.
"""
import dataclasses
import math

import numpy as np
import scipy.linalg as sla

import oracle
import vgtb_synth as vs
from vgtb_synth import systems as S

C = vs.C_LIGHT


def _small_si(mesh=(2, 1, 1), n_electrons=16):
    return vs.diamond_supercell(1, mesh, n_electrons=n_electrons, seed=1001)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_overlap_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    v0 = np.array([-0.007, 0.009, 0.016, -0.004])
    for _ in range(20):
        d = rng.normal(size=3) * 4.0
        r = float(np.linalg.norm(d))
        g = S.sk_block_sp_grad(d, S.bond_integrals(v0, r), S.bond_integrals_dr(v0, r))
        h = 1e-5
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (S.sk_block_sp(d + e, S.bond_integrals(v0, float(np.linalg.norm(d + e)))) -
                  S.sk_block_sp(d - e, S.bond_integrals(v0, float(np.linalg.norm(d - e))))) / (2 * h)
            assert np.abs(g[a] - fd).max() < 1e-9 * max(np.abs(fd).max(), 1e-3)


def test_overlap_gradient_partner_blocks_and_onsite():
    sysm = _small_si()
    key = {}
    for b in range(sysm.n_blocks):
        key[(int(sysm.blk_i[b]), int(sysm.blk_j[b]), *np.round(sysm.blk_d[b], 6))] = b
    for b in range(sysm.n_blocks):
        d = sysm.blk_d[b]
        if np.linalg.norm(d) == 0:
            assert np.all(sysm.blk_ds[b] == 0)
            continue
        p = key[(int(sysm.blk_j[b]), int(sysm.blk_i[b]), *np.round(-d, 6))]
        # S(J, I, -d) = S(I, J, d)^T  =>  its gradient is -(dS/dd)^T (the partner's bond
        # vector is formed separately, so equal to rounding)
        want = -np.transpose(sysm.blk_ds[b], (0, 2, 1))
        assert np.abs(sysm.blk_ds[p] - want).max() < 1e-12 * np.abs(want).max()


def test_momentum_matrix_hermitian_and_time_reversal():
    sysm = _small_si((2, 2, 1))
    for kvec in sysm.kpts:
        p = oracle.overlap_momentum_k(sysm, kvec)
        for a in range(3):
            assert np.abs(p[a] - p[a].conj().T).max() < 1e-15
        # P_{-k} = -conj(P_k) for real two-centre blocks
        pm = oracle.overlap_momentum_k(sysm, -kvec)
        assert np.abs(pm + p.conj()).max() < 1e-15


def test_kick_current_is_the_diamagnetic_closed_form():
    # Ground state on a k-mesh closed under k -> -k: the paramagnetic part
    # sum_k Re Tr(D0 P_k) vanishes, leaving J(0+) = -(A0/c) N_el / Omega.
    sysm = _small_si((2, 2, 2))
    d0, z, _ = oracle.ground_state(sysm)
    a0 = 0.01
    hist, _ = oracle.propagate(sysm, d0, vs.kick_table(1, a0), 0.2, 1, z=z, coupling="momentum")
    j0 = hist["J"][0]
    want = -(a0 / C) * sysm.n_electrons / sysm.volume
    assert abs(j0[0] - want) < 1e-12 * abs(want)
    assert abs(j0[1]) < 1e-12 * abs(want) and abs(j0[2]) < 1e-12 * abs(want)
    # The Peierls current of the same state differs: the two couplings are not the same model.
    hp, _ = oracle.propagate(sysm, d0, vs.kick_table(1, a0), 0.2, 1, z=z)
    assert abs(hp["J"][0][0] - want) > 1e-3 * abs(want)


def test_a_squared_term_is_a_pure_phase():
    sysm = _small_si((2, 1, 1))
    rng = np.random.default_rng(7)
    a = np.array([0.03, -0.02, 0.01])
    for kvec in sysm.kpts:
        s = oracle.overlap_k(sysm, kvec)
        si = oracle.overlap_inverse(s)
        x = rng.normal(size=s.shape) + 1j * rng.normal(size=s.shape)
        d = 0.5 * (x + x.conj().T)
        h_full = oracle.hamiltonian_k(sysm, kvec, a, s, None, "momentum")
        h_lin = h_full - 0.5 * float(a @ a) / C ** 2 * s
        diff = oracle.density_derivative(si, h_full, d) - oracle.density_derivative(si, h_lin, d)
        # Rounding only (the term itself is |A|^2/(2c^2) ~ 7e-8 relative).
        assert np.abs(diff).max() < 1e-13 * np.abs(oracle.density_derivative(si, h_full, d)).max()


def test_orthogonal_basis_has_no_field_dynamics():
    # S = I with no overlap gradient: P = 0 and the |A|^2 term is a phase, so a
    # kicked ground state stays put and carries the constant diamagnetic current.
    sysm = vs.primitive_diamond(kmesh=(2, 2, 2))
    sysm = dataclasses.replace(sysm, blk_ds=np.zeros((sysm.n_blocks, 3, 4, 4)))
    d0, z, _ = oracle.ground_state(sysm)
    a0 = 0.02
    hist, st = oracle.propagate(sysm, d0, vs.kick_table(1, a0), 0.2, 200, z=z, coupling="momentum")
    for ik in range(sysm.n_k):
        assert _rel(st.d_cur[ik], d0[ik]) < 1e-12
    want = -(a0 / C) * sysm.n_electrons / sysm.volume
    assert np.abs(hist["J"][:, 0] - want).max() < 1e-11 * abs(want)


def test_energy_conserved_at_constant_field():
    sysm = _small_si((2, 1, 1))
    d0, z, _ = oracle.ground_state(sysm)
    hist, st = oracle.propagate(sysm, d0, vs.kick_table(1, 0.05), 0.2, 600, z=z,
                                coupling="momentum")
    e = hist["E"]
    assert np.abs(e - e[0]).max() < 1e-6 * abs(e[0])
    assert np.abs(hist["trace"] - sysm.n_electrons).max() < 1e-11
    for d in st.d_cur:
        assert np.abs(d - d.conj().T).max() < 1e-13
    # ... and the field does act: the density moved.
    assert max(_rel(a, b) for a, b in zip(st.d_cur, d0)) > 1e-6


def test_brute_force_matrix_exponential():
    sysm = _small_si((1, 1, 1))
    rng = np.random.default_rng(3)
    a0 = np.array([0.0, 0.03, 0.02])
    x = rng.normal(size=(sysm.n_orb,) * 2) + 1j * rng.normal(size=(sysm.n_orb,) * 2)
    d_start = 0.025 * (x + x.conj().T)
    # H(A) built here from the raw blocks: H0_k + (1/c) A . P_k + |A|^2/(2c^2) S_k,
    # P_k = sum_blocks exp(i k.d) i dS/dd.
    k = sysm.kpts[0]
    n = sysm.n_orb
    s = np.zeros((n, n), complex)
    h = np.zeros((n, n), complex)
    for b in range(sysm.n_blocks):
        i, j = 4 * sysm.blk_i[b], 4 * sysm.blk_j[b]
        ph = np.exp(1j * k @ sysm.blk_d[b])
        s[i:i + 4, j:j + 4] += ph * sysm.blk_s[b]
        h[i:i + 4, j:j + 4] += ph * (sysm.blk_h0[b] + (1j / C) * np.einsum("a,aij->ij", a0, sysm.blk_ds[b]))
    h += 0.5 * (a0 @ a0) / C ** 2 * s
    t_end = 40.0
    u = sla.expm(-1j * np.linalg.solve(s, h) * t_end)
    ref = u @ d_start @ u.conj().T
    errs = []
    for dt in (0.2, 0.1):
        _, st = oracle.propagate(sysm, [d_start], a0[None, :], dt, int(round(t_end / dt)),
                                 coupling="momentum")
        errs.append(_rel(st.d_cur[0], ref))
    assert errs[0] < 0.1
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_work_theorem_under_an_scc_pulse():
    """E(t) - E(0) = Omega int J . E_field dt, E_field = -(1/c) dA/dt, in the
    momentum coupling: dE/dt = sum_k w_k Re Tr(D_k dH/dA) . dA/dt and
    c dH/dA = P_k + (A/c) S_k is the current matrix after Eq. 14, so this ties
    the paramagnetic term P_k of the current to the Hamiltonian of Eq. 12.
    Second order in dt for the leapfrog."""
    sysm = vs.amorphous_si(1, (2, 1, 1), seed=1002, gamma_u=0.25)
    d0, z, _ = oracle.ground_state(sysm)
    errs = []
    for dt in (0.2, 0.1):
        n = int(round(120.0 / dt)) + 1
        T = 100.0
        atab = vs.sin2_pulse_table(n, dt, omega=0.15, duration=T, a_peak=2.0)
        t = np.arange(n) * dt
        env = np.where(t <= T, 1.0, 0.0)
        dadt = env * 2.0 * (math.pi / T * np.sin(2 * math.pi * t / T) * np.cos(0.15 * (t - T / 2))
                            - 0.15 * np.sin(math.pi * t / T) ** 2 * np.sin(0.15 * (t - T / 2)))
        efield = -dadt / C
        hist, _ = oracle.propagate(sysm, d0, atab, dt, n, z=z, coupling="momentum")
        p = sysm.volume * hist["J"][:, 0] * efield
        work = np.concatenate([[0.0], np.cumsum(0.5 * (p[1:] + p[:-1]) * dt)])
        de = hist["E"] - hist["E"][0]
        assert np.abs(de).max() > 1e-5
        errs.append(np.abs(de - work).max() / np.abs(de).max())
    assert errs[0] < 2e-2
    assert 3.0 < errs[0] / errs[1] < 5.0, errs
