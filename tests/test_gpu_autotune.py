"""vgtb_autotune: times the kernel variants, keeps the fastest, leaves the
state alone, and the tuned run agrees with the default one (the variants only
reorder sums).  Covers every precision form on the 64-atom SCC system, a
ragged 13-atom system (N = 52: partial tiles everywhere) and a context on the
small-system path (nothing to tune).
"""
import numpy as np
import pytest

import vgtb_synth as vs

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2308_09782_amd")

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-9, "bf16x3": 1e-8, "fp16x3": 1e-9}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()


def _run(sysm, dt, atab, precision, n, tune, tile=0):
    with pkg.Propagator(sysm, dt, precision, history_capacity=n, tile=tile) as p:
        p.ground_state()
        p.set_field_table(atab)
        tuning = None
        if tune:
            before = p.get_density(0).cpu().numpy()
            tuning = p.autotune(3)
            assert p.step_index == 0
            assert np.array_equal(before, p.get_density(0).cpu().numpy())
        p.step(n)
        h = p.read_observables(0, n)
        d = p.get_density(0).cpu().numpy()
    return h, d, tuning


def _check_tuning(t, precision, norb, np_mult_128):
    assert t["spmm_variant"] in t["spmm_ms"]
    assert t["gemm_tile"] in t["gemm_ms"]
    assert all(v > 0 for v in t["spmm_ms"].values())
    assert all(v > 0 for v in t["gemm_ms"].values())
    want_spmm = ({-1, -2, -4, -11, -12, -14} if norb == 4 else set()) | {1, 2}
    assert set(t["spmm_ms"]) == want_spmm
    if precision in ("bf16x3", "fp16x3"):
        assert set(t["gemm_ms"]) == ({1, 2, 3, 4, 5} if np_mult_128 else {1})
    else:
        assert set(t["gemm_ms"]) == {1, 2, 3}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_autotune_asi64(precision):
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[1500:]
    h0, d0, _ = _run(sysm, c["dt"], atab, precision, 30, False)
    h1, d1, t = _run(sysm, c["dt"], atab, precision, 30, True)
    _check_tuning(t, precision, 4, True)
    jmax = np.abs(h0["J"]).max()
    assert np.abs(h1["J"] - h0["J"]).max() < TOL[precision] * jmax
    err = max(np.linalg.norm(d1[k] - d0[k]) / np.linalg.norm(d0[k]) for k in range(sysm.n_k))
    assert err < TOL[precision]


def test_autotune_ragged():
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    atab = vs.kick_table(1, 0.02)
    h0, d0, _ = _run(sysm, 0.2, atab, "fp64", 40, False)
    h1, d1, t = _run(sysm, 0.2, atab, "fp64", 40, True)
    _check_tuning(t, "fp64", 4, False)
    jmax = np.abs(h0["J"]).max()
    assert np.abs(h1["J"] - h0["J"]).max() < 1e-12 * jmax
    err = max(np.linalg.norm(d1[k] - d0[k]) / np.linalg.norm(d0[k]) for k in range(sysm.n_k))
    assert err < 1e-12


def test_autotune_small_path_has_nothing_to_tune():
    c = vs.CONFIGS["si8_k64"]
    sysm = vs.config_system("si8_k64")
    with pkg.Propagator(sysm, c["dt"], "fp64", history_capacity=4) as p:
        p.ground_state()
        t = p.autotune(2)
    assert t["spmm_ms"] == {} and t["gemm_ms"] == {}


def test_autotune_needs_a_density():
    sysm = vs.config_system("asi64_k8_scc")
    with pkg.Propagator(sysm, 0.2, "fp64", history_capacity=4) as p:
        with pytest.raises(pkg.VgtbError) as ei:
            p.autotune(2)
        assert ei.value.status == 2


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x3"])
def test_split_product_128_tiles_bit_identical(precision):
    # The four 128 x 128 wavefront arrangements (tile_override 2-5) feed every
    # accumulator the same products in the same order: the same bits.
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[1500:]
    runs = {}
    for tile in (2, 3, 4, 5):
        runs[tile] = _run(sysm, c["dt"], atab, precision, 30, False, tile=tile)
    h2, d2, _ = runs[2]
    assert np.abs(h2["J"]).max() > 0
    for tile in (3, 4, 5):
        h, d, _ = runs[tile]
        assert np.array_equal(h2["J"], h["J"]), tile
        assert np.array_equal(d2, d), tile
