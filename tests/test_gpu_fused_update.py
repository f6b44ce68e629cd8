"""The 16-bit split product fused with the leapfrog update (one launch over
mirrored 128 x 128 tile pairs) against the two separate launches: the same
bits for both levels of D and every observable, in the FP16X3 and 3xBF16
forms, over the forward-Euler first step, steps that end in a rescale, a
graph-captured stretch and a non-stationary start (the constant m0 term); on
the 64-atom SCC pulse (N = 256, a 2 x 2 tile grid) with every 128 x 128
wavefront arrangement, and on a ragged 61-atom cell (N = 244 padded to 256:
partial tiles in both the pair and the diagonal units), which is also checked
against the oracle.
"""
import numpy as np
import pytest

import oracle
import vgtb_synth as vs

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2308_09782_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()


def _run(sysm, atab, precision, n, fused, tile, start=None):
    with pkg.Propagator(sysm, 0.2, precision, rescale_every=10, history_capacity=n, tile=tile,
                        fused_update=fused) as p:
        if start is None:
            p.ground_state()
        else:
            p.set_density(start)
        p.set_field_table(atab)
        p.profile(True)
        p.step(7)
        prof = p.profile_read()
        p.profile(False)
        p.step(n - 7)                 # graph replay on the general path
        h = p.read_observables(0, n)
        cur = p.get_density(0).cpu().numpy()
        prev = p.get_density(1).cpu().numpy()
    return h, cur, prev, prof


def _same(a, b):
    for key in ("J", "E", "trace", "q"):
        assert np.array_equal(a[0][key], b[0][key]), key
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x3"])
@pytest.mark.parametrize("tile", [2, 3, 4, 5])
def test_fused_update_bit_identical_asi64(precision, tile):
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[1500:]
    fused = _run(sysm, atab, precision, 40, True, tile)
    plain = _run(sysm, atab, precision, 40, False, tile)
    assert fused[3]["update"][1] == 0 and fused[3]["gemm"][1] == 7
    assert plain[3]["update"][1] == 7
    assert np.abs(fused[0]["J"]).max() > 0
    _same(fused, plain)


def test_fused_update_ragged_nonstationary_against_oracle():
    sysm = vs.random_cell(61, (2, 1, 1), seed=9, gamma_u=0.25)
    assert sysm.n_orb == 244
    d0, z, _ = oracle.ground_state(sysm)
    rng = np.random.default_rng(2)
    start = []
    for d in d0:
        a = rng.normal(size=d.shape) + 1j * rng.normal(size=d.shape)
        start.append(d + 0.003 * (a + a.conj().T))
    start = np.stack(start)
    import dataclasses
    sysm = dataclasses.replace(sysm, z_ref=z)
    atab = vs.kick_table(1, 0.02)
    n = 60
    fused = _run(sysm, atab, "fp16x3", n, True, 2, start=start)
    plain = _run(sysm, atab, "fp16x3", n, False, 2, start=start)
    assert fused[3]["update"][1] == 0
    _same(fused, plain)
    ref, _ = oracle.propagate(sysm, list(start), atab, 0.2, n, z=z)
    jmax = np.abs(ref["J"]).max()
    assert np.abs(fused[0]["J"] - ref["J"]).max() < 1e-5 * jmax
