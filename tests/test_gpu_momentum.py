"""The paper's momentum-matrix coupling (Eq. 12, current matrix P_k + (A/c) S_k)
on the GPU, through the C ABI, against the FP64 oracle's same coupling.

Tolerances as for the Peierls coupling: FP64 density within 1e-10 relative on
both leapfrog levels and the current within 1e-10 of max|J|; 3xBF16 current
within 1e-5 of max|J|.  Plus the closed-form diamagnetic current of a kicked
ground state, J(0+) = -(A0/c) N_el / Omega.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import vgtb_synth as vs

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2308_09782_amd")

pytestmark = pytest.mark.gpu

C = vs.C_LIGHT


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()


def _gpu(sysm, atab, dt, n, precision="fp64", start=None):
    with pkg.Propagator(sysm, dt, precision, history_capacity=n, coupling="momentum") as p:
        if start is None:
            p.ground_state()
        else:
            p.set_density(np.stack(start))
        p.set_field_table(atab)
        p.step(n)
        h = p.read_observables(0, n)
        cur = p.get_density(0).cpu().numpy()
        prev = p.get_density(1).cpu().numpy()
    return h, cur, prev


def _rel_max(a, b):
    return max(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k]) for k in range(len(b)))


def _compare(sysm, atab, dt, n, start=None, z=None, precision="fp64", j_tol=1e-10, rho_tol=1e-10):
    if start is None:
        d_init, z, _ = oracle.ground_state(sysm)
    else:
        d_init = start
    ref, st = oracle.propagate(sysm, d_init, atab, dt, n, z=z, coupling="momentum")
    h, cur, prev = _gpu(sysm, atab, dt, n, precision, start)
    jmax = np.abs(ref["J"]).max()
    assert jmax > 0
    assert np.abs(h["J"] - ref["J"]).max() <= j_tol * jmax
    if rho_tol is not None:
        assert _rel_max(cur, st.d_cur) < rho_tol
        assert _rel_max(prev, st.d_prev) < rho_tol
        assert np.abs(h["E"] - ref["E"]).max() < 1e-11 * np.abs(ref["E"]).max()
        assert np.abs(h["q"] - ref["q"]).max() < 1e-10
    return h, ref


def test_kick_8_atoms_fp64_1000_steps():
    c = vs.CONFIGS["si8_k64"]
    sysm = vs.config_system("si8_k64")
    sysm = sysm.with_kpts(sysm.kpts[::8])
    _compare(sysm, vs.kick_table(1, c["a0"]), c["dt"], 1000)


def test_scc_pulse_64_atoms_fp64_and_split_forms():
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[1500:1900]
    _compare(sysm, atab, c["dt"], 400)
    _compare(sysm, atab, c["dt"], 400, precision="bf16x3", j_tol=1e-5, rho_tol=None)
    _compare(sysm, atab, c["dt"], 400, precision="fp16x3", j_tol=1e-5, rho_tol=None)


def test_ragged_nonstationary_start():
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    d0, z, _ = oracle.ground_state(sysm)
    rng = np.random.default_rng(1)
    start = []
    for d in d0:
        a = rng.normal(size=d.shape) + 1j * rng.normal(size=d.shape)
        start.append(d + 0.005 * (a + a.conj().T))
    sysm = dataclasses.replace(sysm, z_ref=z)
    _compare(sysm, vs.kick_table(1, 0.02), 0.2, 300, start=start, z=z)


def test_kick_current_closed_form():
    sysm = vs.diamond_supercell(1, (2, 2, 2), n_electrons=16, seed=1001)
    a0 = 0.01
    h, _, _ = _gpu(sysm, vs.kick_table(1, a0), 0.2, 2)
    want = -(a0 / C) * sysm.n_electrons / sysm.volume
    assert abs(h["J"][0, 0] - want) < 1e-12 * abs(want)
    assert abs(h["J"][0, 1]) < 1e-12 * abs(want) and abs(h["J"][0, 2]) < 1e-12 * abs(want)
