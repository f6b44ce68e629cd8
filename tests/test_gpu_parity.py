"""GPU path (through the C ABI) against the FP64 oracle, element by element.

Tolerances: FP64 density after the run, max over k of ||D_gpu - D_ref||_F /
||D_ref||_F <= 1e-10 on both leapfrog levels; the current within 1e-10 of
max |J|; energies, traces and charges to near round-off.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import vgtb_synth as vs

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2308_09782_amd")

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()     # fails loudly if the library is missing


def run_gpu(sysm, atab, dt, n_steps, d0=None, precision="fp64", rescale_every=50):
    with pkg.Propagator(sysm, dt, precision, rescale_every=rescale_every,
                        history_capacity=max(n_steps, 1)) as p:
        gap = None
        if d0 is None:
            gap = p.ground_state()
        else:
            p.set_density(np.asarray(d0))
        p.set_field_table(atab)
        p.step(n_steps)
        p.synchronize()
        hist = p.read_observables(0, n_steps) if n_steps else None
        cur = p.get_density(0).cpu().numpy()
        prev = p.get_density(1).cpu().numpy() if n_steps else None
        z = p.reference_charges()
    return dict(hist=hist, cur=cur, prev=prev, z=z, gap=gap)


def rel_max(a, b):
    return max(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k]) for k in range(len(b)))


def _random_hermitian(n, rng, scale=1.0):
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return scale * 0.5 * (a + a.conj().T)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,batch", [(1, 2), (17, 3), (32, 2), (52, 3), (96, 2), (130, 2), (1100, 1)])
def test_zgemm_matches_reference(n, batch):
    rng = np.random.default_rng(n)
    a = rng.normal(size=(batch, n, n)) + 1j * rng.normal(size=(batch, n, n))
    b = rng.normal(size=(batch, n, n)) + 1j * rng.normal(size=(batch, n, n))
    ref = a @ b
    ta = torch.from_numpy(a).cuda()
    tb = torch.from_numpy(b).cuda()
    tc = torch.empty_like(ta)
    pkg.vgtb_zgemm(ta, tb, tc)
    torch.cuda.synchronize()
    c = tc.cpu().numpy()
    for k in range(batch):
        assert np.linalg.norm(c[k] - ref[k]) / np.linalg.norm(ref[k]) < 1e-14 * max(1.0, math.sqrt(n))


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["si8_quarter_degenerate", "random13_scc", "asi64_k8_scc"])
def test_ground_state_matches_oracle(case):
    if case == "si8_quarter_degenerate":
        sysm = vs.diamond_supercell(1, (2, 2, 1), n_electrons=16, seed=1001)
    elif case == "random13_scc":
        sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    else:
        sysm = vs.config_system(case)
    d0, z, gap = oracle.ground_state(sysm)
    g = run_gpu(sysm, np.zeros((1, 3)), 0.2, 0)
    assert rel_max(g["cur"], d0) < 1e-11
    assert np.abs(g["z"] - z).max() < 1e-11
    assert abs(g["gap"] - gap) < 1e-10
    for k in range(sysm.n_k):
        assert np.array_equal(g["cur"][k], g["cur"][k].conj().T)


# ---------------------------------------------------------------------------
def _compare_runs(sysm, atab, dt, n_steps, d0=None, rho_tol=RHO_TOL, j_tol=1e-10):
    if d0 is None:
        d0_ref, z, _ = oracle.ground_state(sysm)
        gpu = run_gpu(sysm, atab, dt, n_steps)
    else:
        d0_ref = d0
        z = np.zeros(sysm.n_atoms) if sysm.z_ref is None else sysm.z_ref
        gpu = run_gpu(sysm, atab, dt, n_steps, d0=np.stack(d0))
    ref, st = oracle.propagate(sysm, d0_ref, atab, dt, n_steps, z=z)
    assert rel_max(gpu["cur"], st.d_cur) < rho_tol
    assert rel_max(gpu["prev"], st.d_prev) < rho_tol
    h = gpu["hist"]
    jmax = np.abs(ref["J"]).max()
    assert np.abs(h["J"] - ref["J"]).max() <= j_tol * max(jmax, 1e-300)
    assert np.abs(h["E"] - ref["E"]).max() < 1e-11 * np.abs(ref["E"]).max()
    assert np.abs(h["trace"] - ref["trace"]).max() < 1e-11 * np.abs(ref["trace"]).max()
    assert np.abs(h["q"] - ref["q"]).max() < 1e-10
    return gpu, ref


def test_c1_si8_k64_kick_1000_steps():
    c = vs.CONFIGS["si8_k64"]
    sysm = vs.config_system("si8_k64")
    _compare_runs(sysm, vs.kick_table(1, c["a0"]), c["dt"], c["n_steps"])


def test_c2_asi64_scc_pulse_1000_steps():
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    n = 1000
    # The first 1000 steps of the 20 fs pulse are too weak to test the drive;
    # start the pulse table at its peak region so that A is large throughout.
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[1500:1500 + n]
    _compare_runs(sysm, atab, c["dt"], n)


def test_ragged_random_cell_scc_nonstationary_start():
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    d0, z, _ = oracle.ground_state(sysm)
    rng = np.random.default_rng(1)
    start = [d + 0.01 * _random_hermitian(sysm.n_orb, rng) for d in d0]
    sysm = dataclasses.replace(sysm, z_ref=z)
    _compare_runs(sysm, vs.kick_table(1, 0.02), 0.2, 300, d0=start)


def test_chain_norb1_current_closed_form():
    a_lat, eps, t, s1, n_k = 4.0, -0.3, -0.1, 0.15, 24
    sysm = vs.linear_chain(n_k, a=a_lat, eps=eps, t=t, s1=s1)
    k = sysm.kpts[:, 0]
    kf = math.pi / (2 * a_lat)
    f = np.where(np.minimum(np.abs(k), np.abs(k - 2 * math.pi / a_lat)) < kf, 2.0, 0.0)
    s_k = 1.0 + 2.0 * s1 * np.cos(k * a_lat)
    d0 = (f / s_k).reshape(n_k, 1, 1).astype(complex)
    dt, n = 0.5, 400
    atab = vs.sin2_pulse_table(n, dt, omega=0.2, duration=150.0, a_peak=30.0)
    g = run_gpu(sysm, atab, dt, n, d0=d0)
    th = (k[None, :] + atab[:, 0:1] / vs.C_LIGHT) * a_lat
    j_ref = -(1.0 / (sysm.volume * n_k)) * np.sum((f / s_k)[None, :] * (-2.0 * t * a_lat * np.sin(th)), axis=1)
    assert np.abs(g["hist"]["J"][:, 0] - j_ref).max() < 1e-12 * np.abs(j_ref).max()


# ---------------------------------------------------------------------------
def test_invariants_exact_hermiticity_trace_energy():
    sysm = vs.diamond_supercell(1, (2, 2, 2), seed=1001)
    g = run_gpu(sysm, vs.kick_table(1, 0.01), 0.2, 400)
    for lev in ("cur", "prev"):
        for k in range(sysm.n_k):
            m = g[lev][k]
            assert np.array_equal(m, m.conj().T)
    h = g["hist"]
    assert np.abs(h["trace"] - sysm.n_electrons).max() < 1e-11
    e = h["E"]
    assert np.abs(e[2::2] - e[0]).max() < 1e-12
    assert np.abs(e[3::2] - e[1]).max() < 1e-12


def test_stationary_ground_state_scc():
    sysm = vs.config_system("asi64_k8_scc")
    g0 = run_gpu(sysm, np.zeros((1, 3)), 0.2, 0)
    g = run_gpu(sysm, np.zeros((1, 3)), 0.2, 200)
    assert rel_max(g["cur"], g0["cur"]) < 1e-12
    assert np.abs(g["hist"]["q"] - g0["z"][None, :]).max() < 1e-11


def test_checkpoint_resume_and_determinism_bitwise():
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    atab = vs.sin2_pulse_table(400, 0.2, 0.1, 60.0, 0.3)
    full = run_gpu(sysm, atab, 0.2, 300)
    again = run_gpu(sysm, atab, 0.2, 300)
    assert np.array_equal(full["cur"], again["cur"])
    with pkg.Propagator(sysm, 0.2, history_capacity=300) as p:
        p.ground_state()
        p.set_field_table(atab)
        p.step(120)
        blob = p.save_state()
    with pkg.Propagator(sysm, 0.2, history_capacity=300) as p:
        p.ground_state()
        p.set_field_table(atab)
        p.load_state(blob)
        assert p.step_index == 120
        p.step(180)
        cur = p.get_density(0).cpu().numpy()
        prev = p.get_density(1).cpu().numpy()
        hist = p.read_observables(120, 180)
    assert np.array_equal(cur, full["cur"])
    assert np.array_equal(prev, full["prev"])
    assert np.array_equal(hist["J"], full["hist"]["J"][120:])


def test_error_paths():
    sysm = vs.config_system("si8_k64")
    with pkg.Propagator(sysm, 0.2, history_capacity=8) as p:
        with pytest.raises(pkg.VgtbError) as ei:
            p.step(1)
        assert ei.value.status == 2                      # VGTB_E_STATE
        p.ground_state()
        p.step(20)
        with pytest.raises(pkg.VgtbError) as ei:
            p.read_observables(0, 20)                    # only the last 8 are kept
        assert ei.value.status == 1
        p.read_observables(12, 8)
        p.step(0)
    with pkg.Propagator(sysm, 5.0) as p:
        with pytest.raises(pkg.VgtbError) as ei:
            p.ground_state()
        assert ei.value.status == 4                      # VGTB_E_UNSTABLE
    bad_s = sysm.blk_s.copy()
    off = np.linalg.norm(sysm.blk_d, axis=1) > 0
    bad_s[off] *= 40.0
    with pytest.raises(pkg.VgtbError) as ei:
        pkg.Propagator(dataclasses.replace(sysm, blk_s=bad_s), 0.2)
    assert ei.value.status == 3                          # VGTB_E_NOT_PD


@pytest.mark.parametrize("case", ["per-step fp64", "per-step fp16x3", "small-path fp64"])
def test_nonfinite_density_is_reported(case):
    # A NaN in the density reaches the trace; synchronising reports
    # VGTB_E_NONFINITE and the context refuses further work.
    if case.startswith("small"):
        sysm, precision = vs.config_system("si8_k64"), "fp64"
    else:
        sysm, precision = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25), case.split()[1]
    with pkg.Propagator(sysm, 0.2, precision, history_capacity=8) as p:
        p.ground_state()
        d = p.get_density(0).cpu().numpy()
        d[0, 3, 3] = np.nan
        p.set_density(d)
        p.set_field_table(vs.kick_table(1, 0.01))
        p.step(2)
        with pytest.raises(pkg.VgtbError) as ei:
            p.synchronize()
        assert ei.value.status == 7                      # VGTB_E_NONFINITE
        with pytest.raises(pkg.VgtbError):
            p.step(1)


# ---------------------------------------------------------------------------
def test_spectrum_matches_oracle():
    """Eqs. 15-16 on the GPU vs the oracle, on a kick run's current and on a
    synthetic damped sinusoid (mean subtraction on and off)."""
    c = vs.CONFIGS["si8_k64"]
    sysm = vs.diamond_supercell(1, (2, 2, 2), seed=1001)
    n = 1500
    g = run_gpu(sysm, vs.kick_table(1, 0.01), 0.2, n)
    j = g["hist"]["J"][:, 0]
    omegas = np.arange(0.005, 0.5, 0.001)
    e0 = -0.01 / vs.C_LIGHT
    with pkg.Propagator(sysm, 0.2) as p:
        sig, eps = p.spectrum(j, 0.2, omegas, e0)
        t = np.arange(4001) * 0.05
        js = np.sin(0.3 * t) * np.exp(-t / 500.0) + 0.1
        sig2, eps2 = p.spectrum(js, 0.05, omegas, 1.0, tau0=150.0, subtract_mean=False)
    ref = oracle.conductivity(j, 0.2, omegas, e0)
    assert np.abs(sig - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(eps - oracle.dielectric(ref, omegas)).max() < 1e-12 * np.abs(eps).max()
    ref2 = oracle.conductivity(js, 0.05, omegas, 1.0, tau0=150.0, subtract_mean=False)
    assert np.abs(sig2 - ref2).max() < 1e-12 * np.abs(ref2).max()
    assert np.imag(eps).max() > 0


@pytest.mark.parametrize("subtract_mean", [True, False])
def test_spectrum_streamed_through_a_small_scratch(subtract_mean):
    """Eqs. 15-16 for a trace and a grid far larger than the context's scratch
    (a 1-atom chain context: 4096 doubles): the trace is cut into about 60
    chunks and the grid into several, with ragged last chunks; the result
    equals the oracle's transform of the whole trace."""
    sysm = vs.linear_chain(2)
    t = np.arange(200003) * 0.05
    js = 0.3 + np.sin(0.31 * t) * np.exp(-t / 5000.0) + 0.2 * np.cos(1.7 * t)
    omegas = np.linspace(0.01, 2.0, 1999)
    with pkg.Propagator(sysm, 0.2) as p:
        sig, eps = p.spectrum(js, 0.05, omegas, 0.7, tau0=3000.0, subtract_mean=subtract_mean)
    ref = oracle.conductivity(js, 0.05, omegas, 0.7, tau0=3000.0, subtract_mean=subtract_mean)
    assert np.abs(sig - ref).max() < 1e-11 * np.abs(ref).max()
    assert np.abs(eps - oracle.dielectric(ref, omegas)).max() < 1e-11 * np.abs(eps).max()


def test_split_k_point_keeps_every_observable():
    """k-weights enter every k-sum: a k-point split into two copies of half its
    weight (a non-uniform mesh of three points) gives the same current, charges
    and energy through an SCC pulse as the two-point mesh, and both match the
    oracle."""
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    kp = np.vstack([sysm.kpts[:1], sysm.kpts[:1], sysm.kpts[1:]])
    kw = np.concatenate([[0.5 * sysm.kw[0]] * 2, sysm.kw[1:]])
    split = sysm.with_kpts(kp, kw)
    atab = vs.sin2_pulse_table(200, 0.2, 0.15, 30.0, 0.4)
    a = run_gpu(sysm, atab, 0.2, 200)["hist"]
    b = run_gpu(split, atab, 0.2, 200)["hist"]
    jmax = np.abs(a["J"]).max()
    assert jmax > 0
    assert np.abs(a["J"] - b["J"]).max() < 1e-12 * jmax
    assert np.abs(a["q"] - b["q"]).max() < 1e-11
    assert np.abs(a["E"] - b["E"]).max() < 1e-11 * np.abs(a["E"]).max()
    d0, z, _ = oracle.ground_state(split)
    ref, _ = oracle.propagate(split, d0, atab, 0.2, 200, z=z)
    assert np.abs(b["J"] - ref["J"]).max() < 1e-10 * jmax
