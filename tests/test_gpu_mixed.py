"""Reduced-precision (deviation-form) GPU propagation against the FP64 oracle.

Bar: the current within 1e-5 of max |J| of the FP64 oracle trajectory; the
density Hermitian bit for bit; Tr(D S) held at N_el by the periodic rescale.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import vgtb_synth as vs

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2308_09782_amd")

pytestmark = pytest.mark.gpu

J_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()


def run_gpu(sysm, atab, dt, n_steps, precision, rescale_every=50, d0=None, **kernel_options):
    with pkg.Propagator(sysm, dt, precision, rescale_every=rescale_every,
                        history_capacity=max(n_steps, 1), **kernel_options) as p:
        if d0 is None:
            p.ground_state()
        else:
            p.set_density(np.asarray(d0))
        p.set_field_table(atab)
        p.step(n_steps)
        p.synchronize()
        hist = p.read_observables(0, n_steps)
        cur = p.get_density(0).cpu().numpy()
        prev = p.get_density(1).cpu().numpy()
    return hist, cur, prev


def j_err(h, ref):
    return np.abs(h["J"] - ref["J"]).max() / np.abs(ref["J"]).max()


def rho_err(cur, dref):
    return max(np.linalg.norm(cur[k] - dref[k]) / np.linalg.norm(dref[k]) for k in range(len(dref)))


@pytest.fixture(scope="module")
def c1_reference():
    c = vs.CONFIGS["si8_k64"]
    sysm = vs.config_system("si8_k64")
    d0, z, _ = oracle.ground_state(sysm)
    atab = vs.kick_table(1, c["a0"])
    ref, st = oracle.propagate(sysm, d0, atab, c["dt"], c["n_steps"], z=z)
    return sysm, atab, c["dt"], c["n_steps"], ref, st


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_c1_mixed_current_within_tolerance(c1_reference, precision):
    sysm, atab, dt, n, ref, st = c1_reference
    h, cur, prev = run_gpu(sysm, atab, dt, n, precision)
    err = j_err(h, ref)
    print(f"{precision}: J err {err:.2e}, rho err {rho_err(cur, st.d_cur):.2e}")
    assert err < J_TOL
    assert rho_err(cur, st.d_cur) < 1e-4
    for k in range(sysm.n_k):
        assert np.array_equal(cur[k], cur[k].conj().T)
        assert np.array_equal(prev[k], prev[k].conj().T)
    assert np.abs(h["trace"] - sysm.n_electrons).max() < 1e-9


@pytest.fixture(scope="module")
def c2_reference():
    """The oracle's 1000 steps of the 64-atom SCC pulse at the pulse peak."""
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    n = 1000
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[1500:1500 + n]
    d0, z, _ = oracle.ground_state(sysm)
    ref, st = oracle.propagate(sysm, d0, atab, c["dt"], n, z=z)
    return sysm, atab, c["dt"], n, ref, st


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_c2_mixed_scc_pulse(c2_reference, precision):
    sysm, atab, dt, n, ref, st = c2_reference
    h, cur, _ = run_gpu(sysm, atab, dt, n, precision)
    err = j_err(h, ref)
    print(f"{precision}: J err {err:.2e}, rho err {rho_err(cur, st.d_cur):.2e}")
    assert err < J_TOL
    assert np.abs(h["q"] - ref["q"]).max() < 1e-5


@pytest.mark.parametrize("precision,tile", [("fp64", 3), ("fp64", 2), ("fp16x3", 2), ("fp16x3", 5),
                                            ("bf16x3", 2)])
def test_c2_scc_pulse_with_the_timed_tiles(c2_reference, precision, tile):
    """The dense-product tiles the benchmark times (FP64: 128 x 64; the split
    forms: 128 x 128 with sixteen wavefronts, fused with the update), forced on
    the 1000-step 64-atom SCC pulse: FP64 density within 1e-10 on both levels
    and current within 1e-10 of max|J|; the split forms' current within 1e-5."""
    sysm, atab, dt, n, ref, st = c2_reference
    with pkg.Propagator(sysm, dt, precision, history_capacity=n, tile=tile) as p:
        p.ground_state()
        p.set_field_table(atab)
        p.step(n)
        h = p.read_observables(0, n)
        cur = p.get_density(0).cpu().numpy()
        prev = p.get_density(1).cpu().numpy()
    err = j_err(h, ref)
    print(f"{precision} tile {tile}: J err {err:.2e}, rho err {rho_err(cur, st.d_cur):.2e}")
    if precision == "fp64":
        assert rho_err(cur, st.d_cur) < 1e-10
        assert rho_err(prev, st.d_prev) < 1e-10
        assert err < 1e-10
        assert np.abs(h["q"] - ref["q"]).max() < 1e-10
    else:
        assert err < J_TOL


@pytest.fixture(scope="module")
def ragged_reference():
    """13 atoms (N = 52: a partial row group of the sparse product, 16-bit planes
    padded to 64), SCC, non-stationary start, 400 steps of the oracle."""
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    d0, z, _ = oracle.ground_state(sysm)
    rng = np.random.default_rng(1)
    start = []
    for d in d0:
        a = rng.normal(size=d.shape) + 1j * rng.normal(size=d.shape)
        start.append(d + 0.002 * (a + a.conj().T))
    sysm = dataclasses.replace(sysm, z_ref=z)
    atab = vs.kick_table(1, 0.02)
    ref, st = oracle.propagate(sysm, start, atab, 0.2, 400, z=z)
    return sysm, np.stack(start), atab, ref, st


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_ragged_padding_and_arbitrary_start(ragged_reference, precision):
    """N = 52 (bf16 planes padded to 64), non-stationary start."""
    sysm, start, atab, ref, st = ragged_reference
    h, cur, _ = run_gpu(sysm, atab, 0.2, 400, precision, d0=start)
    assert j_err(h, ref) < J_TOL
    assert rho_err(cur, st.d_cur) < 1e-4


@pytest.mark.parametrize("variant", [-2, -4, -11, -12, -14])
@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
def test_ragged_deviation_epilogue_every_matrix_core_variant(ragged_reference, precision, variant):
    """The 16-bit planes of W as each matrix-core sparse-product variant writes them
    (C0 subtracted, the rows of an atom gathered across a quad of lanes): a partial
    row group and a column slice mostly beyond N, against the oracle."""
    sysm, start, atab, ref, st = ragged_reference
    h, cur, _ = run_gpu(sysm, atab, 0.2, 400, precision, d0=start, spmm_variant=variant)
    assert j_err(h, ref) < J_TOL
    assert rho_err(cur, st.d_cur) < 1e-4


def _s_chain(n_sites, n_k, seed=11, gamma_u=0.25):
    """One s orbital per site, n_sites sites on a line at perturbed spacing, hopping and
    overlap decaying with distance (second neighbours included), SCC on."""
    rng = np.random.default_rng(seed)
    a = 4.0
    x = a * np.arange(n_sites) + rng.uniform(-0.4, 0.4, n_sites)
    cell = np.diag([a * n_sites, 60.0, 60.0])
    pos = np.stack([x, np.zeros(n_sites), np.zeros(n_sites)], axis=1)

    def hop_h(d):
        return np.array([[-0.1 * np.exp(-(np.linalg.norm(d) - a) / 2.0)]])

    def hop_s(d):
        return np.array([[0.1 * np.exp(-(np.linalg.norm(d) - a) / 2.0)]])

    bi, bj, bd, bh, bs = vs.systems.build_blocks(cell, pos, 1, np.array([[-0.3]]), np.array([[1.0]]),
                                                 hop_h, hop_s, cutoff=9.0)
    k, w = vs.systems.gamma_mesh(cell, (n_k, 1, 1))
    return vs.systems.TBSystem(name="s-chain", cell=cell, pos=pos, norb=1, blk_i=bi, blk_j=bj,
                               blk_d=bd, blk_h0=bh, blk_s=bs, kpts=k, kw=w,
                               n_electrons=float(n_sites),
                               gamma=vs.systems.gamma_matrix(cell, pos, gamma_u), hubbard_u=gamma_u)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_one_orbital_per_atom_reduced_forms(precision):
    # One orbital per atom takes the vector sparse product, whose 16-bit planes
    # are written element by element; N = 40 is padded to 64.
    sysm = _s_chain(40, 4)
    d0, z, _ = oracle.ground_state(sysm)
    sysm = dataclasses.replace(sysm, z_ref=z)
    atab = vs.kick_table(1, 0.02)
    n = 300
    ref, st = oracle.propagate(sysm, d0, atab, 0.2, n, z=z)
    h, cur, _ = run_gpu(sysm, atab, 0.2, n, precision)
    err = j_err(h, ref)
    print(f"{precision} one-orbital chain: J err {err:.2e}, rho err {rho_err(cur, st.d_cur):.2e}")
    assert err < J_TOL
    assert rho_err(cur, st.d_cur) < 1e-4


def test_fp16_split_is_more_accurate_than_bf16():
    # Same product, same matrix-core rate: the scaled fp16 hi/lo split carries
    # about four more bits per part than bf16, so the current error against
    # the oracle drops several-fold.
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    n = 600
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[1500:1500 + n]
    d0, z, _ = oracle.ground_state(sysm)
    ref, _ = oracle.propagate(sysm, d0, atab, c["dt"], n, z=z)
    e_bf = j_err(run_gpu(sysm, atab, c["dt"], n, "bf16x3")[0], ref)
    e_fp = j_err(run_gpu(sysm, atab, c["dt"], n, "fp16x3")[0], ref)
    print(f"J err bf16x3 {e_bf:.2e}, fp16x3 {e_fp:.2e}")
    assert e_fp < e_bf / 4


@pytest.mark.parametrize("small_path,tune", [(True, False), (False, False), (False, True)])
def test_fp16x3_exactly_stationary_when_w_vanishes(small_path, tune):
    # No SCC shift and A = 0: H equals H0 and D stays D(0), so W = H D - H0 D(0)
    # is exactly zero (the same kernel forms both products, also after the
    # autotuner has chosen another sparse product); its maximum is zero, the
    # split keeps scale 1, and the density must stay D(0) bit for bit.  Both the
    # whole-steps kernel of small systems and the per-step kernels.
    sysm = vs.diamond_supercell(1, (2, 2, 2), seed=1001)
    assert sysm.gamma is None
    n = 30
    with pkg.Propagator(sysm, 0.2, "fp16x3", history_capacity=n, small_path=small_path,
                        spmm_variant=2 if tune else 0) as p:
        p.ground_state()
        if tune:
            p.autotune(2)
        d_init = p.get_density(0).cpu().numpy()
        p.set_field_table(vs.kick_table(1, 0.0))
        p.step(n)
        h = p.read_observables(0, n)
        d_end = p.get_density(0).cpu().numpy()
        d_prev = p.get_density(1).cpu().numpy()
    assert np.array_equal(d_end, d_init)
    assert np.array_equal(d_prev, d_init)
    assert np.abs(h["J"]).max() < 1e-13


def test_fp16x3_scale_follows_w_across_a_sudden_kick():
    # 40 steps at A = 0 keep W at rounding level; then A jumps to 0.02 and W's
    # maximum grows by many orders of magnitude in one step, so its per-k scale
    # changes and the planes are split again from the complex64 W.  The whole
    # trajectory must stay within the bar of the FP64 oracle.
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    d0, z, _ = oracle.ground_state(sysm)
    sysm = dataclasses.replace(sysm, z_ref=z)
    n, quiet = 300, 40
    atab = np.zeros((n, 3))
    atab[quiet:, 0] = 0.02
    ref, st = oracle.propagate(sysm, d0, atab, 0.2, n, z=z)
    h, cur, _ = run_gpu(sysm, atab, 0.2, n, "fp16x3")
    err = j_err(h, ref)
    print(f"fp16x3 quiet-then-kick: J err {err:.2e}, rho err {rho_err(cur, st.d_cur):.2e}")
    assert np.abs(ref["J"][:quiet]).max() < 1e-9 * np.abs(ref["J"]).max()
    assert err < J_TOL
    assert rho_err(cur, st.d_cur) < 1e-6


def test_rescale_holds_trace():
    sysm = vs.config_system("asi64_k8_scc")
    c = vs.CONFIGS["asi64_k8_scc"]
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[1500:1900]
    h_on, _, _ = run_gpu(sysm, atab, 0.2, 400, "bf16x3", rescale_every=50)
    h_off, _, _ = run_gpu(sysm, atab, 0.2, 400, "bf16x3", rescale_every=0)
    drift_on = np.abs(h_on["trace"] - sysm.n_electrons)
    drift_off = np.abs(h_off["trace"] - sysm.n_electrons)
    # Right after each rescale the trace is back at N_el to FP64 rounding.
    assert drift_on[50::50].max() < 1e-10
    assert drift_off.max() >= drift_on[50::50].max()


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
def test_mixed_checkpoint_resume_bitwise(precision):
    # fp16x3: the resumed context starts from scale 1, so its first step splits W
    # again with the scale W's maximum calls for; the planes, and so every later
    # step, must be those of the uninterrupted run.
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    atab = vs.sin2_pulse_table(400, 0.2, 0.1, 60.0, 0.3)
    h, full, _ = run_gpu(sysm, atab, 0.2, 300, precision, rescale_every=50)
    with pkg.Propagator(sysm, 0.2, precision, rescale_every=50, history_capacity=300) as p:
        p.ground_state()
        p.set_field_table(atab)
        p.step(130)
        blob = p.save_state()
    with pkg.Propagator(sysm, 0.2, precision, rescale_every=50, history_capacity=300) as p:
        p.ground_state()
        p.set_field_table(atab)
        p.load_state(blob)
        p.step(170)
        cur = p.get_density(0).cpu().numpy()
    assert np.array_equal(cur, full)
