#!/usr/bin/env python3
"""Throughput of the density-matrix propagation on one MI355X.

Workload: the 512-atom amorphous-Si supercell (2048 sp3 orbitals) on the
Gamma-centred 2x2x2 mesh (8 k-points), SCC shift on, 20 fs sin^2 pulse
(omega = 0.1 Ha, peak A = 0.05 au), dt = 0.2 au.  One step = one pass of the
whole hot path over all k-points: observables + Mulliken + SCC shift,
Peierls assembly of the pair blocks, block-sparse H D and dense S^-1 (H D)
on the matrix cores, and the leapfrog update.  Inputs are seeded synthetic stand-ins of
the paper's a-Si structure (no dataset is read).

Prints one JSON line: k-steps/s of the FP16X3 deviation form (three fp16
matrix-core products of power-of-two scaled hi/lo splits; --precision selects
another form) over the timed steps, the same steps in plain FP64 (speed-up and the current's deviation
from the FP64 run), the roofline of the dominant kernel (event-timed inside
the library on the stream it runs on), and the FP64 CPU oracle timed on a
bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "asi512_k8_scc"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "fp16x3": 2500.0}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp16x3", choices=["fp64", "fp32", "bf16x3", "fp16x3"],
                    help="form measured as the headline value (reduced forms propagate the "
                         "deviation from the ground state)")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="skip the FP64 run over the same steps (speed-up and current error)")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--propagator", default="leapfrog", choices=["leapfrog", "crank_nicolson"],
                    help="density leapfrog (Eq. 6, 13) or Crank-Nicolson on the coefficients "
                         "(Eq. 5; FP64 only)")
    ap.add_argument("--coupling", default="peierls", choices=["peierls", "momentum"],
                    help="field coupling: Peierls phase on the H0 blocks, or the momentum "
                         "matrix of the overlap gradients (Eq. 12)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--j-err-steps", type=int, default=1000,
                    help="steps from the ground state over which the headline form's current is "
                         "compared with the FP64 run's (each context keeps stepping after the "
                         "timed and latency steps until it has taken this many)")
    ap.add_argument("--cpu-sample-k", type=int, default=4)
    ap.add_argument("--cpu-sample-steps", type=int, default=6)
    ap.add_argument("--fused-update", action="store_true",
                    help="3xBF16 / FP16X3: the dense product and the leapfrog update as one "
                         "kernel over mirrored tile pairs (VGTB_OPT_FUSE_UPDATE)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel variants instead of timing them first "
                         "(vgtb_autotune)")
    ap.add_argument("--serve", action="store_true",
                    help="instead of timing one workload: serve a seeded Poisson stream of "
                         "propagation requests and report time-to-spectrum p50/p99")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-rate", type=float, default=4.0, help="mean arrivals per second")
    ap.add_argument("--serve-steps", type=int, nargs=2, default=[1000, 10000],
                    help="range of step counts per request")
    ap.add_argument("--serve-precision", default="fp16x3", choices=["fp64", "fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-arena-gib", type=float, default=64.0)
    ap.add_argument("--group", type=int, default=0, metavar="M",
                    help="instead of timing one workload: M seeded 8-atom a-Si cells (2x2x1 mesh) "
                         "stepped as one group (one launch per block of steps for all of them), "
                         "against the same cells stepped one after the other and on M streams")
    ap.add_argument("--group-steps", type=int, default=640)
    ap.add_argument("--group-precision", default="fp16x3", choices=["fp64", "fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--group-scc", action="store_true", help="the cells with the SCC shift (Eq. 10)")
    ap.add_argument("--accuracy", action="store_true",
                    help="instead of timing: run the workload's full step count in the reduced "
                         "forms and in FP64 and report the current and spectrum errors")
    ap.add_argument("--kick", type=float, default=None, metavar="A0",
                    help="drive the workload's system with a delta kick A(t >= 0) = A0 x "
                         "instead of its own drive (accuracy runs: absorption over the whole grid)")
    ap.add_argument("--accuracy-steps", type=int, default=0,
                    help="step count of the accuracy runs (default: the workload's)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed steps, run one plain device copy of this many MiB "
                         "(read N, write N): the reference kernel for hardware byte counters")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_sample(sysm, atab, dt, n_k_sample, n_steps, coupling, propagator):
    """Seconds the oracle takes for n_steps steps of the first n_k_sample k-points."""
    import oracle

    sub = sysm.with_kpts(sysm.kpts[:n_k_sample])
    rng = np.random.default_rng(0)
    n = sysm.n_orb
    d0 = []
    for _ in range(n_k_sample):
        a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        d0.append(1e-3 * 0.5 * (a + a.conj().T))
    z = np.full(sysm.n_atoms, 4.0)
    if propagator == "crank_nicolson":
        ns = n // 2
        c0 = [1e-2 * (rng.normal(size=(n, ns)) + 1j * rng.normal(size=(n, ns))) for _ in range(n_k_sample)]
        cstate = oracle.make_coefficient_state(sub, c0, np.full((n_k_sample, ns), 2.0), z)
        t0 = time.perf_counter()
        oracle.propagate_crank_nicolson(sub, None, None, atab, dt, n_steps, state=cstate, coupling=coupling)
        return time.perf_counter() - t0
    state = oracle.make_state(sub, d0, z)
    t0 = time.perf_counter()
    oracle.propagate(sub, None, atab, dt, n_steps, state=state, coupling=coupling)
    return time.perf_counter() - t0


def cpu_baseline(sysm, atab, dt, n_k_sample, n_steps, coupling="peierls", propagator="leapfrog"):
    """The FP64 oracle as it stands, on a bounded sample of the same workload: with
    the BLAS thread pool at its default (every host thread) and with one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits

    el = _oracle_sample(sysm, atab, dt, n_k_sample, n_steps, coupling, propagator)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        el1 = _oracle_sample(sysm, atab, dt, 1, 1, coupling, propagator)
    return {
        "value": n_k_sample * n_steps / el,
        "unit": "k*steps/s",
        "cores": int(threads),
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "host_threads": os.cpu_count(),
        "sample": f"{n_steps} steps x {n_k_sample} of {sysm.n_k} k-points of the same "
                  f"{sysm.n_orb}-orbital system (numpy/BLAS FP64, {el:.1f} s)",
        "one_thread": {"value": 1.0 / el1, "unit": "k*steps/s", "cores": 1,
                       "sample": f"1 step x 1 k-point, BLAS limited to one thread ({el1:.1f} s)"},
    }


KERNEL_SOURCES = {"fp64": "gemm_mfma.hip", "fp32": "gemm_mfma.hip", "bf16x3": "gemm_split16.hip",
                  "fp16x3": "gemm_split16.hip"}


def counter_traffic(precision, workload):
    """HBM bytes per launch of the dense product from the committed rocprofv3
    counter runs (profiles/traffic.json), or None when they were taken on
    another workload or the kernel's source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_2308_09782_amd", "csrc", KERNEL_SOURCES[precision])
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(precision)
    if not rec or rec.get("workload") != workload:
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("source_sha256") != digest:
        return None
    return rec.get("bytes_per_launch")


def run_form(vg, torch, sysm, atab, dt, precision, warmup, steps, offset, workload, tune=True,
             coupling="peierls", propagator="leapfrog", j_steps=0, fused_update=False):
    """Ground state, warmup, then `steps` timed steps of one precision form, then
    single-step calls for the latency, then more steps (untimed) until j_steps
    steps have been taken; J of every step is returned."""
    total = warmup + steps
    n_lat = min(steps, 20)
    span = max(total + n_lat, j_steps, 1)
    prop = vg.Propagator(sysm, dt, precision, history_capacity=span,
                         coupling=coupling, propagator=propagator, fused_update=fused_update)
    t_init = time.perf_counter()
    gap = prop.ground_state()
    t_init = time.perf_counter() - t_init
    tuning = prop.autotune(5) if tune else None
    prop.set_field_table(atab[offset:])
    prop.step(warmup)
    prop.synchronize()
    prop.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prop.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prop.synchronize()
    prof = prop.profile_read()
    # Latency of single-step calls, after the timed region.
    prop.profile(False)
    events = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat + 1)]
    events[0].record()
    for i in range(n_lat):
        prop.step(1)
        events[i + 1].record()
    torch.cuda.synchronize()
    step_ms = np.array([events[i].elapsed_time(events[i + 1]) for i in range(n_lat)])
    if span > total + n_lat:
        prop.step(span - total - n_lat)
    obs = prop.read_observables(0, span)
    prop_ns = prop.num_states
    prop.close()

    n, nk = sysm.n_orb, sysm.n_k
    gemm_ms, gemm_n = prof["gemm"]
    if propagator == "crank_nicolson":
        # The solve of (S + i dt/2 H) X = S C: factorisation (8/3) N^3 and the
        # forward and back substitution over n_s right-hand sides 8 N^2 n_s, per k.
        ns = prop_ns
        solve_ms = prof["cn_solve"][0]
        launches = max(prof["cn_solve"][1], 1)
        avg_s = solve_ms / launches / 1e3
        flops_per_launch = (8.0 / 3.0 * n ** 3 + 8.0 * n * n * ns) * nk
        achieved = flops_per_launch / avg_s / 1e12
        roof = {"bound": "mfma", "kernel": f"Crank-Nicolson solve (FP64, all {nk} k-points, "
                                           f"{ns} states)",
                "achieved": achieved, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS["fp64"], "traffic": None,
                "flops_per_launch": flops_per_launch, "avg_launch_ms": avg_s * 1e3}
    elif gemm_n:
        gemm_avg_s = gemm_ms / gemm_n / 1e3
        flops_per_launch = 8.0 * n ** 3 * nk
        achieved = flops_per_launch / gemm_avg_s / 1e12
        peak = PEAK_TFLOPS[precision]
        roof = {"bound": "mfma", "kernel": f"dense S^-1 W product ({precision}, all {nk} k-points)",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": counter_traffic(precision, workload) if coupling == "peierls" else None,
                "flops_per_launch": flops_per_launch,
                "avg_launch_ms": gemm_avg_s * 1e3}
        if precision in ("bf16x3", "fp16x3"):
            # three 16-bit products per real product: the matrix cores execute 3x the flops
            roof["mfma_issued_frac"] = 3.0 * achieved / peak
    else:
        # Small systems: whole blocks of steps per launch, FP64 vector arithmetic in LDS.
        sm_ms, sm_n = prof["small"]
        avg_s = sm_ms / max(sm_n, 1) / 1e3
        nnz = len(set(zip(sysm.blk_i.tolist(), sysm.blk_j.tolist()))) * (n // sysm.n_atoms) ** 2
        flops_per_launch = (8.0 * n ** 3 + 8.0 * nnz * n) * nk * steps / max(sm_n, 1)
        achieved = flops_per_launch / avg_s / 1e12
        roof = {"bound": "alu", "kernel": f"whole steps in one launch (FP64, all {nk} k-points)",
                "achieved": achieved, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS["fp64"], "traffic": None,
                "flops_per_launch": flops_per_launch, "avg_launch_ms": avg_s * 1e3}
    kernels = {k: {"avg_ms": (v[0] / v[1] if v[1] else None), "launches": v[1],
                   "share": (v[0] / max(sum(x[0] for x in prof.values()), 1e-30))}
               for k, v in prof.items() if v[1]}
    return {
        "value": nk * steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "roofline": roof,
        "step_latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                            "p99": float(np.percentile(step_ms, 99)), "max": float(step_ms.max())},
        "kernels": kernels,
        "init_s": t_init,
        "autotune": tuning,
        "min_gap_ha": gap,
        "trace_drift": float(np.abs(obs["trace"] - sysm.n_electrons).max()),
        "J": obs["J"],
        "steps_taken": span,
    }


def accuracy_run(vg, torch, sysm, atab, dt, forms, n_steps, workload):
    """Full-length runs of each form from the ground state: J(t) over the whole run and
    the spectra of Eqs. 15-16 (computed on the GPU), reduced forms against FP64."""
    c_light = 137.035999084
    omegas = np.linspace(0.02, 0.30, 281)
    # E(t) = -(1/c) dA/dt of the drive, transformed like the current (Eq. 15 with E0 = 1).
    ax = atab[:n_steps, 0] if atab.shape[0] >= n_steps else np.concatenate(
        [atab[:, 0], np.full(n_steps - atab.shape[0], atab[-1, 0])])
    ef = -np.gradient(ax, dt) / c_light
    runs = {}
    for prec in forms:
        with vg.Propagator(sysm, dt, prec, history_capacity=n_steps) as prop:
            prop.ground_state()
            prop.set_field_table(atab)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prop.step(n_steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            obs = prop.read_observables(0, n_steps)
            jt, _ = prop.spectrum(obs["J"][:, 0], dt, omegas, 1.0)
            if atab.shape[0] == 1:      # kick: E(t) = -(A0/c) delta(t)
                et = np.full(omegas.size, -atab[0, 0] / c_light, dtype=np.complex128)
            else:
                et, _ = prop.spectrum(ef, dt, omegas, 1.0, subtract_mean=False)
        runs[prec] = {"J": obs["J"][:, 0], "trace": obs["trace"], "jw": jt, "ew": et,
                      "value": sysm.n_k * n_steps / el, "seconds": el}
        print(f"accuracy run: {prec} done in {el:.1f} s", file=sys.stderr, flush=True)
    ref = runs["fp64"]
    band = np.abs(ref["ew"]) >= 0.1 * np.abs(ref["ew"]).max()
    def absorption(r):
        return 4.0 * np.pi * np.real(r["jw"][band] / r["ew"][band]) / omegas[band]
    a_ref = absorption(ref)
    jmax = np.abs(ref["J"]).max()

    def peaks(a, m=3):
        """The m largest local maxima of the absorption in the band (their omega, Ha)."""
        w = omegas[band]
        idx = [i for i in range(1, a.size - 1) if a[i] >= a[i - 1] and a[i] > a[i + 1]]
        return sorted(float(w[i]) for i in sorted(idx, key=lambda i: -a[i])[:m])
    out = {"metric": f"accuracy of the reduced forms against FP64, full {n_steps}-step run",
           "workload": workload, "steps": n_steps, "dt": dt,
           "omega_band_ha": [float(omegas[band].min()), float(omegas[band].max())],
           "fp64": {"k_steps_per_s": ref["value"], "seconds": ref["seconds"],
                    "trace_drift": float(np.abs(ref["trace"] - sysm.n_electrons).max()),
                    "peak_omega_ha": float(omegas[np.argmax(np.abs(ref["jw"]))]),
                    "absorption_peak_omega_ha": float(omegas[band][np.argmax(a_ref)]),
                    "absorption_peaks_ha": peaks(a_ref)}}
    for prec in forms:
        if prec == "fp64":
            continue
        r = runs[prec]
        a = absorption(r)
        ip = np.argmax(np.abs(ref["jw"]))
        out[prec] = {
            "k_steps_per_s": r["value"], "seconds": r["seconds"],
            "j_err_max_over_run": float(np.abs(r["J"] - ref["J"]).max() / jmax),
            "trace_drift": float(np.abs(r["trace"] - sysm.n_electrons).max()),
            "current_spectrum_err": float(np.abs(r["jw"] - ref["jw"]).max() / np.abs(ref["jw"]).max()),
            "peak_omega_ha": float(omegas[np.argmax(np.abs(r["jw"]))]),
            "peak_height_rel_err": float(abs(abs(r["jw"][ip]) - abs(ref["jw"][ip])) / abs(ref["jw"][ip])),
            "absorption_err_in_band": float(np.abs(a - a_ref).max() / np.abs(a_ref).max()),
            "absorption_peak_omega_ha": float(omegas[band][np.argmax(a)]),
            "absorption_peaks_ha": peaks(a),
        }
    return out


def serve_run(vg, args):
    """A seeded Poisson stream of requests: a-Si/c-Si-shaped systems of 8-512 atoms,
    meshes from Gamma to 4x4x4, sin^2 pulses with omega in [0.05, 0.3] Ha, 1000-10000
    steps, the FP16X3 form by default; served by vgtb_server_run with admission by arena
    footprint.  Every request must succeed: a failed one is reported and makes the run
    exit non-zero."""
    import vgtb_synth as vs
    rng = np.random.default_rng(1005)
    n = args.serve_requests
    gaps = rng.exponential(1.0 / args.serve_rate, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    # (atoms, meshes allowed, weight): large systems on coarse meshes only.
    kinds = [(8, [(1, 1, 1), (2, 2, 2), (4, 4, 4)], 0.4), (64, [(1, 1, 1), (2, 2, 2), (4, 4, 4)], 0.35),
             (216, [(1, 1, 1), (2, 2, 2)], 0.15), (512, [(1, 1, 1), (2, 2, 2)], 0.10)]
    cache = {}
    omegas = np.linspace(0.02, 0.30, 57)
    reqs = []
    for i in range(n):
        atoms, meshes, _ = kinds[rng.choice(len(kinds), p=[k[2] for k in kinds])]
        mesh = meshes[rng.integers(len(meshes))]
        key = (atoms, mesh)
        if key not in cache:
            ncell = {8: 1, 64: 2, 216: 3, 512: 4}[atoms]
            cache[key] = (vs.diamond_supercell(1, mesh) if atoms == 8 else
                          vs.amorphous_si(ncell, mesh, gamma_u=0.25))
        steps = int(rng.integers(args.serve_steps[0], args.serve_steps[1] + 1))
        omega = float(rng.uniform(0.05, 0.30))
        dt = 0.2
        field = vs.sin2_pulse_table(steps, dt, omega, 0.5 * steps * dt, 0.05)
        reqs.append(dict(system=cache[key], dt=dt, precision=args.serve_precision, n_steps=steps,
                         field=field, arrival_s=float(arrivals[i]), omegas=omegas))
    with vg.Server(int(args.serve_arena_gib * 2 ** 30), max_active=args.serve_slots) as srv:
        res, summ = srv.run(reqs)
    ok = [x for x in res if x["status"] == 0]
    failed = [{"request": i, "status": x["status"], "message": x["message"]}
              for i, x in enumerate(res) if x["status"] != 0]
    if not ok:
        return {"metric": "serving", "requests": n, "completed": 0, "failed": failed}
    tts = np.array([x["finished_s"] - x["arrival_s"] for x in ok])
    wait = np.array([x["admitted_s"] - x["arrival_s"] for x in ok])
    mix = {}
    for r in reqs:
        k = f"{r['system'].n_atoms} atoms x {r['system'].n_k} k"
        mix[k] = mix.get(k, 0) + 1
    return {
        "metric": "serving: time-to-spectrum p50/p99 (s) and aggregate k*steps/s",
        "requests": n, "completed": len(ok), "failed": failed, "rate_per_s": args.serve_rate,
        "steps_range": list(args.serve_steps), "slots": args.serve_slots,
        "arena_gib": args.serve_arena_gib, "dtype": f"{args.serve_precision} products, f64 state",
        "time_to_spectrum_s": {"p50": float(np.percentile(tts, 50)), "p99": float(np.percentile(tts, 99)),
                               "max": float(tts.max())},
        "admission_wait_s": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
        "k_steps_per_s": summ["k_steps_per_s"], "makespan_s": summ["makespan_s"],
        "peak_active": summ["peak_active"], "peak_gib": summ["peak_bytes"] / 2 ** 30,
        "mix": mix,
        "data": "synthetic (seeded a-Si/c-Si supercells, sin^2 pulses, Poisson arrivals)",
    }


def group_run(vg, torch, args):
    """M small systems (8-atom a-Si cells of different seeds, 4 k-points each) under
    sin^2 pulses of different frequencies: k*steps/s when stepped as one group,
    one after the other on one stream, and each on its own stream."""
    import vgtb_synth as vs
    m, steps, warm = args.group, args.group_steps, 64
    gu = 0.25 if args.group_scc else None
    cells = [vs.amorphous_si(1, (2, 2, 1), seed=3000 + i, gamma_u=gu) for i in range(m)]
    fields = [vs.sin2_pulse_table(warm + steps, 0.2, 0.05 + 0.25 * i / max(m - 1, 1), 100.0, 0.05)
              for i in range(m)]
    kst = sum(c.n_k for c in cells) * steps

    def open_all(streams=None):
        props = []
        for i, c in enumerate(cells):
            ctx = torch.cuda.stream(streams[i]) if streams else torch.cuda.stream(torch.cuda.current_stream())
            with ctx:
                p = vg.Propagator(c, 0.2, args.group_precision, history_capacity=warm + steps)
                p.ground_state()
                p.set_field_table(fields[i])
            props.append(p)
        torch.cuda.synchronize()
        return props

    out = {}
    props = open_all()
    with vg.Group(props) as g:
        g.step(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        out["grouped"] = time.perf_counter() - t0
    j_group = [p.read_observables(warm, steps)["J"] for p in props]
    for p in props:
        p.close()
    props = open_all()
    for p in props:
        p.step(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in props:
        p.step(steps)
    torch.cuda.synchronize()
    out["one_stream"] = time.perf_counter() - t0
    same = all(np.array_equal(p.read_observables(warm, steps)["J"], j) for p, j in zip(props, j_group))
    for p in props:
        p.close()
    streams = [torch.cuda.Stream() for _ in range(m)]
    props = open_all(streams)
    for p in props:
        p.step(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in props:
        p.step(steps)
    torch.cuda.synchronize()
    out["m_streams"] = time.perf_counter() - t0
    for p in props:
        p.close()
    return {
        "metric": "group of small systems: k*steps/s", "unit": "k*steps/s", "systems": m,
        "k_points_each": 4, "atoms_each": 8, "steps": steps, "scc": bool(args.group_scc),
        "dtype": args.group_precision,
        "value": kst / out["grouped"],
        "one_stream": kst / out["one_stream"], "m_streams": kst / out["m_streams"],
        "grouped_equals_alone": bool(same),
        "data": "synthetic (seeded 8-atom a-Si cells, sin^2 pulses of different frequencies)",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the propagation runs on a single GPU; it is not sharded across GPUs)",
              file=sys.stderr)
        return 2
    import torch
    import vgtb_synth as vs
    import paper_2308_09782_amd as vg

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    if args.group:
        print(json.dumps(group_run(vg, torch, args)), flush=True)
        return 0
    if args.serve:
        rec = serve_run(vg, args)
        print(json.dumps(rec), flush=True)
        return 1 if rec["failed"] else 0
    cfg = vs.CONFIGS[args.workload]
    sysm = vs.config_system(args.workload)
    dt = cfg["dt"]
    if args.kick is not None:
        atab = vs.kick_table(1, args.kick)
    elif cfg["drive"] == "pulse":
        atab = vs.sin2_pulse_table(cfg["n_steps"], dt, cfg["omega"], cfg["t_fs"] * vs.FS_AU, cfg["a_peak"])
    else:
        atab = vs.kick_table(1, cfg["a0"])
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.accuracy:
        forms = ["fp64", "bf16x3", "fp16x3", "fp32"]
        label = args.workload + (f", kick A0 = {args.kick}" if args.kick is not None else "")
        print(json.dumps(accuracy_run(vg, torch, sysm, atab, dt, forms,
                                      args.accuracy_steps or cfg["n_steps"], label)), flush=True)
        return 0
    total = args.warmup + args.steps
    # Warmup and timed steps sit in the middle of the pulse, where A is large.
    offset = min(2000, max(0, atab.shape[0] - total))
    if args.propagator == "crank_nicolson":
        args.precision = "fp64"
    compare = args.precision != "fp64" and not args.no_fp64_compare
    j_steps = args.j_err_steps if compare else 0
    head = run_form(vg, torch, sysm, atab, dt, args.precision, args.warmup, args.steps, offset,
                    args.workload, tune=not args.no_autotune, coupling=args.coupling,
                    propagator=args.propagator, j_steps=j_steps,
                    fused_update=args.fused_update)
    print(f"timed {args.precision}: {head['value']:.1f} k*steps/s", file=sys.stderr, flush=True)
    ref = None
    if compare:
        ref = run_form(vg, torch, sysm, atab, dt, "fp64", args.warmup, args.steps, offset,
                       args.workload, tune=not args.no_autotune, coupling=args.coupling,
                       j_steps=j_steps)
        print(f"timed fp64: {ref['value']:.1f} k*steps/s", file=sys.stderr, flush=True)

    n, nk = sysm.n_orb, sysm.n_k
    out = {
        "metric": "k*steps/s (512-atom a-Si, 2048 orbitals, 8 k-points), mixed vs FP64",
        "value": head["value"],
        "unit": "k*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 products, f64 state",
                  "bf16x3": "bf16x3 products, f64 state",
                  "fp16x3": "fp16x3 products, f64 state"}[args.precision],
        "data": "synthetic (seeded a-Si supercell, sp3 Slater-Koster blocks, sin^2 pulse)",
        "config": {"workload": f"{args.workload}: {sysm.n_atoms}-atom a-Si, {n} orbitals, "
                               f"{nk} k-points (2x2x2), SCC, sin^2 pulse, dt={dt}",
                   "n_orb": n, "n_k": nk, "n_atoms": sysm.n_atoms, "precision": args.precision,
                   "coupling": args.coupling, "propagator": args.propagator,
                   "fused_update": args.fused_update,
                   "parallelism": "single GPU, all k-points batched"},
        "roofline": head["roofline"],
        "step_latency_ms": head["step_latency_ms"],
        "kernels": head["kernels"],
        "init_s": head["init_s"],
        "autotune": head["autotune"],
        "min_gap_ha": head["min_gap_ha"],
        "trace_drift": head["trace_drift"],
        "cpu_baseline": None,
    }
    if ref is not None:
        jr, jm = ref["J"][:, 0], head["J"][:, 0]
        out["fp64"] = {k: ref[k] for k in ("value", "ms_per_step", "roofline", "step_latency_ms", "kernels",
                                            "autotune")}
        out["speedup_vs_fp64"] = head["value"] / ref["value"]
        out["j_err_vs_fp64"] = float(np.abs(jm - jr).max() / np.abs(jr).max())
        out["j_err_steps"] = int(min(head["steps_taken"], ref["steps_taken"]))
        out["j_err_window"] = (f"steps {offset}..{offset + out['j_err_steps'] - 1} of the pulse, "
                               "both forms from the ground state")
    if not args.no_cpu_baseline:
        print("timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sysm, atab[offset:], dt, args.cpu_sample_k, args.cpu_sample_steps,
                                           args.coupling, args.propagator)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
