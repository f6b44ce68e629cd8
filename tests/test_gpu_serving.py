"""Serving (vgtb_server_*): requests of different sizes, k-meshes, pulses and
precision forms arrive over time, are admitted by arena footprint into a few
slots, overlap on the GPU, and each result (J(t) and the spectrum of
Eqs. 15-16) equals the one computed alone, bit for bit.  Two requests are
also checked against the oracle: J(t) of an FP64 kick within 1e-10 of its
maximum and of an FP16X3 pulse within 1e-5, and a 5000-step Gamma-only
request, whose spectrum is streamed through a small context scratch.
"""
import numpy as np
import pytest

import oracle
import vgtb_synth as vs

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2308_09782_amd")

pytestmark = pytest.mark.gpu

OMEGAS = np.linspace(0.02, 0.3, 57)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()


def _pulse(n, omega, a_peak=0.05):
    return vs.sin2_pulse_table(n, 0.2, omega, 0.6 * n * 0.2, a_peak)


def _requests():
    si8 = vs.config_system("si8_k64")
    si8_8k = si8.with_kpts(si8.kpts[:8])
    si8_g = si8.with_kpts(si8.kpts[:1], np.ones(1))
    r13 = vs.random_cell(13, (2, 1, 1), seed=3, gamma_u=0.25)
    r9 = vs.random_cell(9, (1, 1, 1), seed=5)
    a64 = vs.config_system("asi64_k8_scc")
    return [
        dict(system=si8_8k, dt=0.2, precision="bf16x3", n_steps=200, field=_pulse(200, 0.1),
             arrival_s=0.0),
        dict(system=r13, dt=0.2, precision="fp64", n_steps=300, field=vs.kick_table(1, 0.02),
             arrival_s=0.0, e0=-0.02 / 137.035999084),
        dict(system=a64, dt=0.2, precision="fp16x3", n_steps=150, field=_pulse(150, 0.2),
             arrival_s=0.0),
        dict(system=si8, dt=0.2, precision="fp64", n_steps=256, field=vs.kick_table(1, 0.01),
             arrival_s=0.1, e0=-0.01 / 137.035999084),
        dict(system=r9, dt=0.2, precision="fp16x3", n_steps=400, field=_pulse(400, 0.15),
             arrival_s=0.1),
        dict(system=a64, dt=0.2, precision="fp64", n_steps=100, field=_pulse(100, 0.15),
             arrival_s=0.0),
        dict(system=si8_g, dt=0.2, precision="fp16x3", n_steps=5000, field=vs.kick_table(1, 0.01),
             arrival_s=0.05, e0=-0.01 / 137.035999084),
    ]


def _alone(r):
    # A server context launches every step directly; graphs give the same bits.
    with pkg.Propagator(r["system"], r["dt"], r["precision"], history_capacity=r["n_steps"],
                        graphs=False) as p:
        p.ground_state()
        p.set_field_table(r["field"])
        p.step(r["n_steps"])
        j = p.read_observables(0, r["n_steps"])["J"]
        sig, _ = p.spectrum(j[:, 0], r["dt"], OMEGAS, r.get("e0", 1.0), 200.0)
    return j, sig


def _ws(r):
    return pkg.vgtb_workspace_size(r["system"], pkg.make_options(r["dt"], r["precision"], 50,
                                                                 r["n_steps"]))


def test_mix_equals_alone_and_admission_by_footprint():
    reqs = _requests()
    for r in reqs:
        r["omegas"] = OMEGAS
    sizes = [_ws(r) for r in reqs]
    # Room for the largest request and half the next: the two 64-atom requests
    # (both arriving at once) can never be resident together.
    order = np.argsort(sizes)
    big1, big2 = int(order[-1]), int(order[-2])
    budget = sizes[big1] + sizes[big2] // 2
    print(f"serving {len(reqs)} requests in {budget} bytes, 3 slots", flush=True)
    with pkg.Server(budget, max_active=3) as srv:
        res, summ = srv.run(reqs)
    print(f"served: makespan {summ['makespan_s']:.2f} s", flush=True)
    assert all(x["status"] == 0 for x in res), [(x["status"], x["message"]) for x in res]
    assert summ["peak_bytes"] <= budget
    assert 1 <= summ["peak_active"] <= 3
    assert summ["k_steps"] == sum(r["system"].n_k * r["n_steps"] for r in reqs)
    for r, x, ws in zip(reqs, res, sizes):
        assert x["workspace_bytes"] == ws
        assert x["arrival_s"] <= x["admitted_s"] <= x["ready_s"] <= x["finished_s"]
    # Admission by footprint: whenever a request is admitted, the requests then
    # resident (admitted earlier, not yet finished) fit in the arena with it.
    for i, x in enumerate(res):
        resident = [j for j, y in enumerate(res)
                    if y["admitted_s"] <= x["admitted_s"] < y["finished_s"]]
        assert i in resident
        assert sum(sizes[j] for j in resident) <= budget
    first, second = sorted((big1, big2), key=lambda i: res[i]["admitted_s"])
    assert res[second]["admitted_s"] >= res[first]["finished_s"]
    for i, (r, x) in enumerate(zip(reqs, res)):
        j, sig = _alone(r)
        print(f"request {i}: alone run done", flush=True)
        assert np.array_equal(x["J"], j)
        assert np.array_equal(x["sigma"], sig)
        assert np.abs(j).max() > 0
    # Against the oracle: the FP64 kick (1e-10) and the FP16X3 pulse (1e-5).
    for i, bar in ((1, 1e-10), (4, 1e-5)):
        r = reqs[i]
        d0, z, _ = oracle.ground_state(r["system"])
        ref, _ = oracle.propagate(r["system"], d0, r["field"], r["dt"], r["n_steps"], z=z)
        jmax = np.abs(ref["J"]).max()
        err = np.abs(res[i]["J"] - ref["J"]).max() / jmax
        print(f"request {i} ({r['precision']}) J vs oracle: {err:.2e}", flush=True)
        assert err < bar
    # The long Gamma-only request: its spectrum against the oracle's transform of
    # the same current (the context scratch holds 4096 doubles: many chunks).
    g = reqs[6]
    sig_ref = oracle.conductivity(res[6]["J"][:, 0], g["dt"], OMEGAS, g["e0"], 200.0)
    assert np.abs(res[6]["sigma"] - sig_ref).max() < 1e-11 * np.abs(sig_ref).max()


def test_oversized_and_invalid_requests_fail_alone():
    reqs = _requests()[:3]
    sizes = [_ws(r) for r in reqs]
    budget = sorted(sizes)[1] + 1024          # the largest one cannot fit
    bad = dict(reqs[0], n_steps=0)
    with pkg.Server(budget, max_active=2) as srv:
        res, summ = srv.run(reqs + [bad])
    big = int(np.argmax(sizes))
    for i, x in enumerate(res[:3]):
        assert x["status"] == (5 if i == big else 0)
        if i == big:
            assert x["slot"] == -1
            assert "exceeds the arena" in x["message"]
        else:
            assert x["message"] == ""
    assert res[3]["status"] == 1
    assert "n_steps" in res[3]["message"]
    assert summ["k_steps"] == sum(r["system"].n_k * r["n_steps"] for i, r in enumerate(reqs) if i != big)
