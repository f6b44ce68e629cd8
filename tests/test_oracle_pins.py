"""Pins of the FP64 oracle against facts fixed by mathematics, not by the oracle.

Each test checks one piece of the oracle against a closed form, a textbook
special case, brute-force matrix-exponential propagation, an exact
invariant, or a value printed in the paper, so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails at least one.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import vgtb_synth as vs

HERE = os.path.dirname(os.path.abspath(__file__))


def _small_si(nk_mesh=(2, 1, 1), seed=1001, n_electrons=16):
    return vs.diamond_supercell(1, nk_mesh, n_electrons=n_electrons, seed=seed)


def _random_hermitian(n, rng, scale=1.0):
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return scale * 0.5 * (a + a.conj().T)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------------------
# P1: closed-form leapfrog solution for a constant Hamiltonian (any start).
# ---------------------------------------------------------------------------
def test_p1_leapfrog_closed_form():
    sysm = _small_si()
    rng = np.random.default_rng(7)
    dt, n_steps = 0.2, 1000
    a0 = np.array([0.01, 0.0, 0.0])
    d0 = [_random_hermitian(sysm.n_orb, rng, 0.05) for _ in range(sysm.n_k)]
    _, st = oracle.propagate(sysm, d0, a0[None, :], dt, n_steps)
    for ik, kvec in enumerate(sysm.kpts):
        # Independent eigen-solution of the generalised problem in the test.
        s = np.zeros((sysm.n_orb, sysm.n_orb), complex)
        h = np.zeros_like(s)
        kk = kvec + a0 / vs.C_LIGHT
        for b in range(sysm.n_blocks):
            i, j = sysm.blk_i[b], sysm.blk_j[b]
            sl_i = slice(4 * i, 4 * i + 4)
            sl_j = slice(4 * j, 4 * j + 4)
            s[sl_i, sl_j] += np.exp(1j * kvec @ sysm.blk_d[b]) * sysm.blk_s[b]
            h[sl_i, sl_j] += np.exp(1j * kk @ sysm.blk_d[b]) * sysm.blk_h0[b]
        eps, c = sla.eigh(h, s)
        cinv = np.linalg.inv(c)
        b0 = cinv @ d0[ik] @ cinv.conj().T
        om = eps[:, None] - eps[None, :]
        x1 = b0 - 1j * dt * om * b0
        root = np.sqrt(1.0 - (om * dt) ** 2)
        l1 = -1j * om * dt + root
        l2 = -1j * om * dt - root
        # x_j = a l1^j + b l2^j with x_0 = b0, x_1 = x1.
        a = (x1 - l2 * b0) / (l1 - l2)
        bb = b0 - a
        for level, nj in ((st.d_cur[ik], n_steps), (st.d_prev[ik], n_steps - 1)):
            bn = a * l1 ** nj + bb * l2 ** nj
            ref = c @ bn @ c.conj().T
            assert _rel(level, ref) < 5e-12


# ---------------------------------------------------------------------------
# P2: brute force exp(-i S^-1 H t) D0 exp(+i H S^-1 t); O(dt^2) convergence.
# ---------------------------------------------------------------------------
def test_p2_expm_and_second_order():
    sysm = _small_si((1, 1, 1))
    rng = np.random.default_rng(3)
    a0 = np.array([0.0, 0.02, 0.01])
    d0 = [_random_hermitian(sysm.n_orb, rng, 0.05)]
    t_end = 40.0
    kk = sysm.kpts[0] + a0 / vs.C_LIGHT
    s = np.zeros((sysm.n_orb, sysm.n_orb), complex)
    h = np.zeros_like(s)
    for b in range(sysm.n_blocks):
        i, j = sysm.blk_i[b], sysm.blk_j[b]
        s[4 * i:4 * i + 4, 4 * j:4 * j + 4] += sysm.blk_s[b] * np.exp(1j * sysm.kpts[0] @ sysm.blk_d[b])
        h[4 * i:4 * i + 4, 4 * j:4 * j + 4] += sysm.blk_h0[b] * np.exp(1j * kk @ sysm.blk_d[b])
    u = sla.expm(-1j * np.linalg.solve(s, h) * t_end)
    ref = u @ d0[0] @ u.conj().T
    errs = []
    for dt in (0.2, 0.1):
        n = int(round(t_end / dt))
        _, st = oracle.propagate(sysm, d0, a0[None, :], dt, n)
        errs.append(_rel(st.d_cur[0], ref))
    assert errs[0] < 0.1
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, ratio


# ---------------------------------------------------------------------------
# P3: invariants: Hermiticity, Tr(D_k S_k) per k, even/odd energy.
# ---------------------------------------------------------------------------
def test_p3_invariants_constant_field():
    sysm = _small_si((2, 1, 1))
    d0, z, _ = oracle.ground_state(sysm)
    hist, st = oracle.propagate(sysm, d0, vs.kick_table(1, 0.01), 0.2, 400, z=z)
    for ik in range(sysm.n_k):
        d = st.d_cur[ik]
        assert np.abs(d - d.conj().T).max() < 1e-13
        s = oracle.overlap_k(sysm, sysm.kpts[ik])
        assert abs(np.trace(d @ s).real - sysm.n_electrons) < 1e-11
    e = hist["E"]
    # E_{n+1} = E_{n-1}: the even and the odd subsequences are each constant.
    assert np.abs(e[2::2] - e[0]).max() < 1e-12
    assert np.abs(e[3::2] - e[1]).max() < 1e-12
    assert np.abs(hist["trace"] - sysm.n_electrons).max() < 1e-11


# ---------------------------------------------------------------------------
# P4: stationarity of the ground state at zero field (also with SCC).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scc", [False, True])
def test_p4_ground_state_stationary(scc):
    if scc:
        sysm = vs.amorphous_si(1, (2, 1, 1), seed=1002, gamma_u=0.25)
    else:
        sysm = _small_si((2, 2, 1))     # quarter filling: degenerate Fermi groups occur
    d0, z, _ = oracle.ground_state(sysm)
    _, st = oracle.propagate(sysm, d0, np.zeros((1, 3)), 0.2, 100, z=z)
    for ik in range(sysm.n_k):
        assert _rel(st.d_cur[ik], d0[ik]) < 1e-12
        # Idempotency of the ground state in the S metric (f = 2): D S D = 2 D
        # holds for a non-degenerate Fermi level.
    q = oracle.mulliken(sysm, d0, [oracle.overlap_k(sysm, k) for k in sysm.kpts])
    assert abs(q.sum() - sysm.n_electrons) < 1e-10


def test_p4_ground_state_projector_half_filling():
    sysm = vs.diamond_supercell(1, (2, 1, 1), seed=1001)   # 32 electrons, gapped
    d0, z, gap = oracle.ground_state(sysm)
    assert gap > 1e-4
    for ik, kvec in enumerate(sysm.kpts):
        s = oracle.overlap_k(sysm, kvec)
        assert _rel(d0[ik] @ s @ d0[ik], 2.0 * d0[ik]) < 1e-12


# ---------------------------------------------------------------------------
# P5: time reversibility of the leapfrog scheme.
# ---------------------------------------------------------------------------
def test_p5_reversibility():
    sysm = _small_si((2, 1, 1))
    rng = np.random.default_rng(11)
    d0 = [_random_hermitian(sysm.n_orb, rng, 0.05) for _ in range(sysm.n_k)]
    a = vs.kick_table(1, 0.01)
    n = 200
    _, st = oracle.propagate(sysm, d0, a, 0.2, n)
    st.d_prev, st.d_cur = st.d_cur, st.d_prev
    _, st = oracle.propagate(sysm, None, a, -0.2, n - 1, state=st)
    for ik in range(sysm.n_k):
        assert _rel(st.d_cur[ik], d0[ik]) < 1e-11


# ---------------------------------------------------------------------------
# P6: gauge identity and dH/dA by finite differences.
# ---------------------------------------------------------------------------
def test_p6_momentum_is_derivative_of_h():
    sysm = vs.amorphous_si(1, (2, 1, 1), seed=1005, gamma_u=None)
    kvec = sysm.kpts[1]
    a = np.array([0.03, -0.02, 0.05])
    h = 1e-3
    pi = oracle.momentum_k(sysm, kvec, a)
    for alpha in range(3):
        e = np.zeros(3)
        e[alpha] = h
        fd = (oracle.h0_k(sysm, kvec, a + e) - oracle.h0_k(sysm, kvec, a - e)) / (2 * h)
        # c dH/dA = Pi; central difference error O(h^2 |d|^3 / c^3)
        assert np.abs(fd * vs.C_LIGHT - pi[alpha]).max() < 1e-8 * np.abs(pi[alpha]).max() + 1e-12


def test_p6_gauge_identity_trajectory():
    """A constant A at k gives the same D(t) as A = 0 at the shifted k + A/c
    when the overlap is the same (S = I system)."""
    sysm = vs.primitive_diamond(kmesh=(2, 1, 1))
    a0 = np.array([0.5, 0.2, -0.1])
    rng = np.random.default_rng(5)
    d0 = [_random_hermitian(sysm.n_orb, rng, 0.1) for _ in range(sysm.n_k)]
    _, st1 = oracle.propagate(sysm, d0, a0[None, :], 0.2, 50)
    shifted = sysm.with_kpts(sysm.kpts + a0 / vs.C_LIGHT, sysm.kw)
    _, st2 = oracle.propagate(shifted, d0, np.zeros((1, 3)), 0.2, 50)
    for ik in range(sysm.n_k):
        assert _rel(st1.d_cur[ik], st2.d_cur[ik]) < 1e-13
    # H itself: phase on every block vs shifted k.
    for kvec in sysm.kpts:
        h1 = oracle.h0_k(sysm, kvec, a0)
        h2 = oracle.h0_k(sysm, kvec + a0 / vs.C_LIGHT, np.zeros(3))
        assert np.abs(h1 - h2).max() < 1e-15


# ---------------------------------------------------------------------------
# P7: textbook models.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("s1", [0.0, 0.15])
def test_p7_chain_current_closed_form(s1):
    a_lat, eps, t = 4.0, -0.3, -0.1
    n_k = 24
    sysm = vs.linear_chain(n_k, a=a_lat, eps=eps, t=t, s1=s1)
    k = sysm.kpts[:, 0]
    kf = math.pi / (2 * a_lat)
    f = np.where(np.minimum(np.abs(k), np.abs(k - 2 * math.pi / a_lat)) < kf, 2.0, 0.0)
    s_k = 1.0 + 2.0 * s1 * np.cos(k * a_lat)                   # unphased overlap
    d0 = [np.array([[f[i] / s_k[i]]], complex) for i in range(n_k)]
    dt, n = 0.5, 400
    atab = vs.sin2_pulse_table(n, dt, omega=0.2, duration=150.0, a_peak=30.0)
    hist, st = oracle.propagate(sysm, d0, atab, dt, n)
    omega_vol = sysm.volume
    th = (k[None, :] + atab[:, 0:1] / vs.C_LIGHT) * a_lat
    dhdk = -2.0 * t * a_lat * np.sin(th)
    j_ref = -(1.0 / (omega_vol * n_k)) * np.sum((f / s_k)[None, :] * dhdk, axis=1)
    assert np.abs(hist["J"][:, 0] - j_ref).max() < 1e-13 * max(np.abs(j_ref).max(), 1e-30) + 1e-18
    assert np.abs(j_ref).max() > 1e-8
    assert np.abs(hist["J"][:, 1:]).max() == 0.0
    for i in range(n_k):
        assert abs(st.d_cur[i][0, 0] - d0[i][0, 0]) < 1e-13


def test_p7_sp3_diamond_gamma_levels():
    vh = vs.systems.V_NOMINAL
    sysm = vs.primitive_diamond(vh=vh)
    h = oracle.h0_k(sysm, np.zeros(3), np.zeros(3))
    ev = np.sort(np.linalg.eigvalsh(h))
    es, ep = vs.systems.EPS_S, vs.systems.EPS_P
    vss, vsp, vpps, vppp = vh
    ref = np.sort([es + 4 * vss, es - 4 * vss] + [ep + 4.0 / 3.0 * (vpps + 2 * vppp)] * 3
                  + [ep - 4.0 / 3.0 * (vpps + 2 * vppp)] * 3)
    assert np.abs(ev - ref).max() < 1e-14
    # At X = 2 pi / a (1, 0, 0) the four nearest-neighbour phases cancel for s-s.
    hx = oracle.h0_k(sysm, np.array([2 * math.pi / vs.systems.A_SI, 0, 0]), np.zeros(3))
    assert abs(hx[0, 4]) < 1e-14
    assert abs(hx[4, 0]) < 1e-14


def test_p7_s_identity_reduces_to_commutator():
    sysm = vs.primitive_diamond(kmesh=(1, 1, 1))
    rng = np.random.default_rng(2)
    d = _random_hermitian(8, rng)
    h = oracle.h0_k(sysm, sysm.kpts[0], np.array([0.1, 0, 0]))
    s_inv = oracle.overlap_inverse(oracle.overlap_k(sysm, sysm.kpts[0]))
    assert np.abs(s_inv - np.eye(8)).max() == 0.0
    ddot = oracle.density_derivative(s_inv, h, d)
    assert np.abs(1j * ddot - (h @ d - d @ h)).max() < 1e-14


# ---------------------------------------------------------------------------
# P8: SCC pieces.
# ---------------------------------------------------------------------------
def test_p8_hubbard_limit_by_hand():
    sysm = vs.primitive_diamond(kmesh=(1, 1, 1))     # S = I, 2 atoms
    rng = np.random.default_rng(4)
    d = _random_hermitian(8, rng, 0.3) + 2.0 * np.eye(8)
    u = 0.4
    gamma = u * np.eye(2)
    z = np.array([4.0, 4.0])
    s = np.eye(8, dtype=complex)
    q = oracle.mulliken(sysm, [d], [s])
    q_hand = np.array([d[0:4, 0:4].trace().real, d[4:8, 4:8].trace().real])
    assert np.allclose(q, q_hand, rtol=0, atol=1e-14)
    v = oracle.scc_potential(gamma, q, z)
    assert np.allclose(v, u * (q_hand - z), atol=1e-14)
    h = oracle.hamiltonian_k(sysm, sysm.kpts[0], np.zeros(3), s, v)
    h0 = oracle.h0_k(sysm, sysm.kpts[0], np.zeros(3))
    shift = np.diag(np.repeat(u * (q_hand - z), 4))
    assert np.abs((h - h0) - shift).max() < 1e-14


def test_p8_mulliken_sum_rule_and_energy_conservation_scc():
    sysm = vs.amorphous_si(1, (2, 1, 1), seed=1002, gamma_u=0.25)
    d0, z, _ = oracle.ground_state(sysm)
    rng = np.random.default_rng(9)
    # Perturb the start (Hermitian) so that the SCC dynamics is non-trivial.
    dd = [d + 0.01 * _random_hermitian(sysm.n_orb, rng) for d in d0]
    hist, _ = oracle.propagate(sysm, dd, np.zeros((1, 3)), 0.1, 600, z=z)
    tr = hist["trace"]
    assert np.abs(hist["q"].sum(axis=1) - tr).max() < 1e-10
    e = hist["E"]
    assert np.abs(e - e[0]).max() < 2e-4 * np.abs(e[0])
    # No secular drift: the late-time mean stays where the early-time mean was.
    assert abs(e[-100:].mean() - e[:100].mean()) < 1e-6


def test_p8_work_theorem_scc():
    """E(t) - E(0) = Omega * int J . E_field dt with E_field = -(1/c) dA/dt."""
    sysm = vs.amorphous_si(1, (2, 1, 1), seed=1002, gamma_u=0.25)
    d0, z, _ = oracle.ground_state(sysm)
    errs = []
    for dt in (0.2, 0.1):
        t_end = 120.0
        n = int(round(t_end / dt)) + 1
        T = 100.0
        atab = vs.sin2_pulse_table(n, dt, omega=0.15, duration=T, a_peak=2.0)
        t = np.arange(n) * dt
        env = np.where(t <= T, 1.0, 0.0)
        dadt = env * 2.0 * (math.pi / T * np.sin(2 * math.pi * t / T) * np.cos(0.15 * (t - T / 2))
                            - 0.15 * np.sin(math.pi * t / T) ** 2 * np.sin(0.15 * (t - T / 2)))
        efield = -dadt / vs.C_LIGHT
        hist, _ = oracle.propagate(sysm, d0, atab, dt, n, z=z)
        p = sysm.volume * hist["J"][:, 0] * efield
        work = np.concatenate([[0.0], np.cumsum(0.5 * (p[1:] + p[:-1]) * dt)])
        de = hist["E"] - hist["E"][0]
        assert np.abs(de).max() > 1e-5
        errs.append(np.abs(de - work).max() / np.abs(de).max())
    assert errs[0] < 2e-2
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


# ---------------------------------------------------------------------------
# P9: spectrum closed forms, linearity and passivity.
# ---------------------------------------------------------------------------
def test_p9_filtered_transform_closed_form():
    om0, dt, n, tau = 0.3, 0.01, 40001, 200.0
    t = np.arange(n) * dt
    j = np.sin(om0 * t)
    omegas = np.array([0.1, 0.25, 0.3, 0.45])
    sig = oracle.conductivity(j, dt, omegas, e0=1.0, tau0=tau, subtract_mean=False)
    T = t[-1]
    ref = []
    for om in omegas:
        def prim(x, w):
            # int exp(((i w) - 1/tau) x) dx
            a = 1j * w - 1.0 / tau
            return np.exp(a * x) / a
        val = (prim(T, om + om0) - prim(0, om + om0) - prim(T, om - om0) + prim(0, om - om0)) / (2j)
        ref.append(val)
    assert np.abs(sig - np.array(ref)).max() < 1e-5 * np.abs(ref).max()


def test_p9_linearity_passivity_and_symmetry():
    sysm = vs.diamond_supercell(1, (2, 2, 2), seed=1001)     # 32 e, gapped, cubic
    d0, z, _ = oracle.ground_state(sysm)
    dt, n = 0.2, 1500
    h1, _ = oracle.propagate(sysm, d0, vs.kick_table(1, 0.005), dt, n, z=z)
    h2, _ = oracle.propagate(sysm, d0, vs.kick_table(1, 0.010), dt, n, z=z)
    j1, j2 = h1["J"][:, 0], h2["J"][:, 0]
    assert np.abs(j2 - 2 * j1).max() < 1e-3 * np.abs(j2).max()
    # P10: cubic crystal, A along x: no transverse current.
    assert np.abs(h2["J"][:, 1:]).max() < 1e-12 * np.abs(j2).max()
    omegas = np.arange(0.05, 0.5, 0.005)
    e0 = -0.01 / vs.C_LIGHT
    im = oracle.absorption(j2, dt, omegas, e0)
    assert im.max() > 0
    assert im.min() > -0.05 * im.max()


def test_p9_mean_subtraction_removes_a_constant_current():
    """Eq. 15 with the mean removed (Section 3): a constant plus a sinusoid
    sampled over whole periods gives the transform of the sinusoid alone."""
    dt, n, tau = 0.01, 40000, 200.0
    om0 = 2.0 * math.pi * 19 / (n * dt)        # 19 whole periods in the n samples
    t = np.arange(n) * dt
    j = 0.37 + np.sin(om0 * t)
    omegas = np.array([0.1, 0.25, om0, 0.45])
    sig = oracle.conductivity(j, dt, omegas, e0=1.0, tau0=tau, subtract_mean=True)
    T = t[-1]

    def prim(x, w):
        a = 1j * w - 1.0 / tau
        return np.exp(a * x) / a

    ref = np.array([(prim(T, om + om0) - prim(0, om + om0) - prim(T, om - om0) + prim(0, om - om0)) / (2j)
                    for om in omegas])
    assert np.abs(sig - ref).max() < 1e-5 * np.abs(ref).max()
    # Without the subtraction the constant adds about 0.37 / (1/tau - i omega),
    # at least 0.37 / 0.45 = 0.82 in magnitude on this grid.
    raw = oracle.conductivity(j, dt, omegas, e0=1.0, tau0=tau, subtract_mean=False)
    assert np.abs(raw - ref).min() > 0.5


def test_p9_drude_dielectric_of_a_free_electron_current():
    """Eq. 16 against the Drude form.  With S = I and no overlap gradient the
    momentum coupling (Eq. 12) leaves a kicked ground state unchanged, so the
    current is the constant diamagnetic one, J = -(A0/c) N_el / Omega.  With
    E0 = -A0/c, Eq. 15 (no mean removed) tends to sigma = n_e / (1/tau0 - i w),
    n_e = N_el / Omega, and Eq. 16 to the damped free-electron dielectric
    function eps = 1 - w_p^2 / (w^2 + i w / tau0), w_p^2 = 4 pi n_e."""
    import dataclasses
    sysm = vs.primitive_diamond(kmesh=(2, 2, 2))
    sysm = dataclasses.replace(sysm, blk_ds=np.zeros((sysm.n_blocks, 3, 4, 4)))
    d0, z, _ = oracle.ground_state(sysm)
    a0, dt, tau = 0.02, 0.2, 20.0
    n = int(round(20 * tau / dt)) + 1           # exp(-20) of the filter is left at the end
    hist, _ = oracle.propagate(sysm, d0, vs.kick_table(1, a0), dt, n, z=z, coupling="momentum")
    jx = hist["J"][:, 0]
    n_e = sysm.n_electrons / sysm.volume
    assert np.abs(jx + (a0 / vs.C_LIGHT) * n_e).max() < 1e-11 * (a0 / vs.C_LIGHT) * n_e
    omegas = np.array([0.05, 0.12, 0.3, 0.61, 1.0])
    e0 = -a0 / vs.C_LIGHT
    sig = oracle.conductivity(jx, dt, omegas, e0, tau0=tau, subtract_mean=False)
    eps = oracle.dielectric(sig, omegas)
    wp2 = 4.0 * math.pi * n_e
    drude = 1.0 - wp2 / (omegas ** 2 + 1j * omegas / tau)
    # The trapezoid rule is off by (dt |i w - 1/tau|)^2 / 12 relative (Euler-Maclaurin).
    tol = (dt * np.abs(1j * omegas - 1.0 / tau)) ** 2 / 12.0 * 1.5 + 1e-8
    assert np.all(np.abs(eps - drude) <= tol * np.abs(drude - 1.0)), (eps, drude)
    assert np.all(eps.imag > 0.0)
    # Well below the plasma frequency the free-electron gas screens: Re eps < 0.
    assert eps[0].real < 0.0 and eps[-1].real > 0.0


def test_k_weights_enter_every_k_sum():
    """A k-point split into two copies of half its weight is the same mesh:
    the current (Eq. 14), the charges and the energy do not change, through an
    SCC pulse."""
    sysm = vs.amorphous_si(1, (2, 1, 1), seed=1002, gamma_u=0.25)
    kp = np.vstack([sysm.kpts[:1], sysm.kpts[:1], sysm.kpts[1:]])
    kw = np.concatenate([[0.5 * sysm.kw[0]] * 2, sysm.kw[1:]])
    split = sysm.with_kpts(kp, kw)
    atab = vs.sin2_pulse_table(120, 0.2, 0.15, 20.0, 0.5)
    outs = []
    for s_ in (sysm, split):
        d0, z, _ = oracle.ground_state(s_)
        hist, _ = oracle.propagate(s_, d0, atab, 0.2, 120, z=z)
        outs.append(hist)
    a, b = outs
    assert np.abs(a["J"]).max() > 1e-6
    assert np.abs(a["J"] - b["J"]).max() < 1e-12 * np.abs(a["J"]).max()
    assert np.abs(a["q"] - b["q"]).max() < 1e-11
    assert np.abs(a["E"] - b["E"]).max() < 1e-11 * np.abs(a["E"]).max()


def test_p10_gamma_point_real_and_zero_current():
    sysm = vs.amorphous_si(1, (1, 1, 1), seed=1002, gamma_u=None)
    d0, z, _ = oracle.ground_state(sysm)
    h = oracle.h0_k(sysm, np.zeros(3), np.zeros(3))
    assert np.abs(h.imag).max() == 0.0
    assert np.abs(d0[0].imag).max() < 1e-13
    jc, _, _, _ = oracle.observables(sysm, d0, [oracle.overlap_k(sysm, np.zeros(3))], np.zeros(3), z)
    assert np.abs(jc).max() < 1e-14


# ---------------------------------------------------------------------------
# Values the paper prints (tests/golden/paper_parameters.json).
# ---------------------------------------------------------------------------
def test_golden_paper_parameters():
    g = json.load(open(os.path.join(HERE, "golden", "paper_parameters.json")))
    # Default filter of the spectrum routine is the paper's tau0.
    import inspect
    assert inspect.signature(oracle.conductivity).parameters["tau0"].default == g["filter_tau0_au"]["value"]
    # 18000 steps of 0.002 fs = 36 fs (Table 1 caption).
    assert abs(g["table1_steps"]["value"] * g["time_step_fs"]["value"] - g["table1_total_fs"]["value"]) < 1e-9
    # 1e12 W/cm^2 <-> E0 ~ 0.274 eV/A: I = E^2 * 3.50944758e16 W/cm^2 (E in a.u.).
    e_au = math.sqrt(g["laser_intensity_W_cm2"]["value"] / 3.50944758e16)
    e_v_per_a = e_au * 51.4220674763
    assert abs(e_v_per_a - g["laser_E0_eV_per_A"]["value"]) < g["laser_E0_eV_per_A"]["rel_tol"] * 0.274
    # 20 fs in atomic time.
    assert abs(g["laser_duration_fs"]["value"] * vs.FS_AU - 826.827) < 1e-2


def test_column_derivative_equals_full():
    """The column-sampled Eq. 6 agrees with the full one (used at full size)."""
    sysm = _small_si((1, 1, 1))
    rng = np.random.default_rng(8)
    d = _random_hermitian(sysm.n_orb, rng)
    s = oracle.overlap_k(sysm, sysm.kpts[0])
    h = oracle.h0_k(sysm, sysm.kpts[0], np.array([0.02, 0.0, 0.01]))
    si = oracle.overlap_inverse(s)
    cols = [0, 5, 31]
    full = oracle.density_derivative(si, h, d)
    assert np.abs(oracle.density_derivative_columns(si, h, d, cols) - full[:, cols]).max() < 1e-14
    # the derivative of a Hermitian density is Hermitian
    assert np.abs(full - full.conj().T).max() < 1e-13


def test_occupations_by_hand():
    """Aufbau with a degenerate group straddling the Fermi level (equal sharing)."""
    eps = np.array([0.3, -1.0, 0.0, 0.0, 0.0, 2.0])
    f = oracle.occupations(eps, 5.0)
    assert np.allclose(f, [0.0, 2.0, 1.0, 1.0, 1.0, 0.0])
    f = oracle.occupations(np.array([-1.0, 0.0, 1e-10, 1.0]), 4.0)
    assert np.allclose(f, [2.0, 1.0, 1.0, 0.0])
    assert oracle.occupations(np.array([-1.0, 0.0]), 0.0).sum() == 0.0
