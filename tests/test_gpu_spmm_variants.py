"""Every kernel variant of the block-sparse product W = H D propagates alike.

The product runs as vector FMAs (one or two columns per thread) or on the
FP64 matrix cores (one, two or four 16-column slices per wave, with four real
products per complex one, or three: Dr Hr, Di Hi and (Dr + Di)(Hr + Hi)), over
row groups of 4, 8 or 16 atoms; the variants agree to rounding.
Each variant is checked against the oracle on a ragged 13-atom system (a
partial row group and a partial column slice) from a non-stationary start,
and against the default variant on the 64-atom a-Si pulse case in the FP64
and 3xBF16 forms.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import vgtb_synth as vs

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2308_09782_amd")

pytestmark = pytest.mark.gpu

VARIANTS = [
    {},
    {"spmm_variant": 1},
    {"spmm_variant": 1, "spmm_group": 4},
    {"spmm_variant": 2},
    {"spmm_variant": 2, "spmm_group": 4},
    {"spmm_variant": -2},
    {"spmm_variant": -4, "spmm_group": 4},
    {"spmm_variant": -1, "spmm_group": 16},
    {"spmm_variant": -2, "spmm_group": 16},
    {"spmm_variant": -11},
    {"spmm_variant": -14},
    {"spmm_variant": -12, "spmm_group": 4},
    {"spmm_variant": -14, "spmm_group": 16},
]
IDS = ["default"] + ["-".join(f"{k[5:]}{v}" for k, v in c.items()) for c in VARIANTS[1:]]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()


def _run(variant, sysm, dt, atab, n_steps, start=None, precision="fp64"):
    with pkg.Propagator(sysm, dt, precision, history_capacity=n_steps, **variant) as p:
        if start is None:
            p.ground_state()
        else:
            p.set_density(start)
        p.set_field_table(atab)
        p.step(n_steps)
        hist = p.read_observables(0, n_steps)
        cur = p.get_density(0).cpu().numpy()
        prev = p.get_density(1).cpu().numpy()
    return hist, cur, prev


@pytest.fixture(scope="module")
def ragged_case():
    sysm = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    d0, z, _ = oracle.ground_state(sysm)
    rng = np.random.default_rng(5)
    start = []
    for d in d0:
        a = rng.normal(size=d.shape) + 1j * rng.normal(size=d.shape)
        start.append(d + 0.005 * (a + a.conj().T))
    sysm = dataclasses.replace(sysm, z_ref=z)
    atab = vs.kick_table(1, 0.02)
    n = 150
    ref, st = oracle.propagate(sysm, start, atab, 0.2, n, z=z)
    return sysm, np.stack(start), atab, n, ref, st


@pytest.mark.parametrize("variant", VARIANTS, ids=IDS)
def test_variant_matches_oracle_ragged(ragged_case, variant):
    sysm, start, atab, n, ref, st = ragged_case
    hist, cur, prev = _run(variant, sysm, 0.2, atab, n, start=start)
    for got, want in ((cur, st.d_cur), (prev, st.d_prev)):
        err = max(np.linalg.norm(got[k] - want[k]) / np.linalg.norm(want[k]) for k in range(sysm.n_k))
        assert err < 1e-10
    jmax = np.abs(ref["J"]).max()
    assert np.abs(hist["J"] - ref["J"]).max() <= 1e-10 * jmax


@pytest.fixture(scope="module")
def asi64_case():
    c = vs.CONFIGS["asi64_k8_scc"]
    sysm = vs.config_system("asi64_k8_scc")
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    return sysm, c["dt"], full[1500:1560], 60


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3", 1e-8), ("fp16x3", 1e-8)])
def test_variants_agree_asi64(asi64_case, precision, tol):
    sysm, dt, atab, n = asi64_case
    base_h, base_d, _ = _run(VARIANTS[0], sysm, dt, atab, n, precision=precision)
    jmax = np.abs(base_h["J"]).max()
    assert jmax > 0
    for variant in VARIANTS[1:]:
        h, d, _ = _run(variant, sysm, dt, atab, n, precision=precision)
        dj = np.abs(h["J"] - base_h["J"]).max() / jmax
        dd = max(np.linalg.norm(d[k] - base_d[k]) / np.linalg.norm(base_d[k]) for k in range(sysm.n_k))
        assert dj < tol, (variant, dj)
        assert dd < tol, (variant, dd)
