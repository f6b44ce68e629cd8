"""vgtb_spectrum_noalloc (no context, no allocation: a fixed device scratch per
GPU) against the context entry point vgtb_spectrum and the oracle, through the
C ABI, on two calls in a row - a long trace and a large grid that stream
through the scratch in several chunks, then a smaller one - plus its argument
checks."""
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


def _inputs():
    t = np.arange(200003) * 0.05
    big = (0.3 + np.sin(0.31 * t) * np.exp(-t / 5000.0) + 0.2 * np.cos(1.7 * t), 0.05,
           np.linspace(0.01, 2.0, 1999), 0.7, 3000.0)
    rng = np.random.default_rng(11)
    small = (np.cumsum(rng.normal(size=1500)) * 1e-6, 0.2, np.arange(0.005, 0.5, 0.0087),
             -0.01 / vs.C_LIGHT, 200.0)
    return big, small


def test_noalloc_spectrum_equals_the_context_entry_point():
    sysm = vs.linear_chain(2)
    runs = []
    for j, dt, om, e0, tau in _inputs():          # the second call is smaller
        for sub in (True, False):
            sig, eps = pkg.spectrum_noalloc(j, dt, om, e0, tau, subtract_mean=sub)
            with pkg.Propagator(sysm, 0.2) as p:
                sig_c, eps_c = p.spectrum(j, dt, om, e0, tau, subtract_mean=sub)
            ref = oracle.conductivity(j, dt, om, e0, tau0=tau, subtract_mean=sub)
            scale = np.abs(ref).max()
            assert np.abs(sig - sig_c).max() < 1e-12 * scale
            assert np.abs(eps - eps_c).max() < 1e-12 * np.abs(eps_c).max()
            assert np.abs(sig - ref).max() < 1e-11 * scale
            runs.append(sig)
    assert runs[0].shape != runs[2].shape


def test_noalloc_spectrum_rejects_bad_arguments():
    lib = pkg.load_library()
    j = np.zeros(10)
    om = np.array([0.1, 0.0])
    out = np.zeros(2, dtype=np.complex128)
    st = lib.vgtb_spectrum_noalloc(10, j.ctypes.data, 0.2, 2, om.ctypes.data, 1.0, 200.0, 1,
                                   out.ctypes.data, None, None)
    assert st == pkg.VGTB_E_INVAL
    assert b"nonzero" in lib.vgtb_last_error(None)
    st = lib.vgtb_spectrum_noalloc(1, j.ctypes.data, 0.2, 1, om.ctypes.data, 1.0, 200.0, 1,
                                   out.ctypes.data, None, None)
    assert st == pkg.VGTB_E_INVAL
    st = lib.vgtb_spectrum_noalloc((1 << 30) + 1, j.ctypes.data, 0.2, 1, om.ctypes.data, 1.0, 200.0, 1,
                                   out.ctypes.data, None, None)
    assert st == pkg.VGTB_E_INVAL
    assert b"2^30" in lib.vgtb_last_error(None)
