"""Graph replay of the per-step launches gives bit-identical results.

Pairs of steps are replayed from graphs captured once per leapfrog parity;
the forward-Euler first step, the steps that end in a rescale and odd leftovers
are launched directly, so every run below interleaves replays with direct
work.  Each run is repeated with graphs turned off (the VGTB_OPT_NO_GRAPHS option) and the two
must agree bit for bit: the history (J, E, Tr, q) and both density levels.
The runs change the field table mid-run (the device field ring is refilled),
reload a checkpoint (the device step counter is reset) and start from a
non-stationary density (the captured update carries the constant m0 term).
"""
import numpy as np
import pytest

import vgtb_synth as vs

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2308_09782_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()


@pytest.fixture(scope="module")
def case():
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    return sysm, c["dt"], full


def _run(graphs, sysm, dt, full, precision, start=None):
    out = {}
    with pkg.Propagator(sysm, dt, precision, rescale_every=10, history_capacity=400,
                        graphs=graphs) as p:
        if start is None:
            p.ground_state()
        else:
            p.set_density(start)
        p.set_field_table(full[1500:])
        for n in (1, 2, 7, 30, 1, 40):
            p.step(n)
        blob = p.save_state()
        p.set_field_table(full[2000:])          # new table mid-run
        for n in (33, 64, 5):
            p.step(n)
        out["h1"] = p.read_observables(0, p.step_index)
        out["d1"] = p.get_density(0).cpu().numpy()
        p.load_state(blob)                       # back to step 81
        p.set_field_table(full[1500:])
        p.step(70)
        out["h2"] = p.read_observables(0, p.step_index)
        out["d2"] = p.get_density(0).cpu().numpy()
        out["p2"] = p.get_density(1).cpu().numpy()
    return out


def _same(a, b):
    for key in ("d1", "d2", "p2"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("h1", "h2"):
        for q in ("J", "E", "trace", "q"):
            assert np.array_equal(a[key][q], b[key][q]), (key, q)


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "fp16x3"])
def test_graph_replay_bit_identical(case, precision):
    sysm, dt, full = case
    with_graphs = _run(True, sysm, dt, full, precision)
    without = _run(False, sysm, dt, full, precision)
    assert np.abs(with_graphs["h1"]["J"]).max() > 0
    _same(with_graphs, without)


def test_graph_replay_nonstationary_start(case):
    sysm, dt, full = case
    rng = np.random.default_rng(4)
    with pkg.Propagator(sysm, dt, "fp64", history_capacity=1) as p:
        p.ground_state()
        d0 = p.get_density(0).cpu().numpy()
    a = rng.normal(size=d0.shape) + 1j * rng.normal(size=d0.shape)
    start = d0 + 0.002 * (a + np.conj(np.swapaxes(a, 1, 2)))
    with_graphs = _run(True, sysm, dt, full, "bf16x3", start=start)
    without = _run(False, sysm, dt, full, "bf16x3", start=start)
    _same(with_graphs, without)
