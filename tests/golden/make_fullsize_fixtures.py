"""Write the oracle fixtures of the two large workloads (calls only oracle/
and the seeded input generator; nothing here comes from the GPU library).

  asi512_k8_scc_pulse30.npz - the 512-atom a-Si cell (2048 orbitals, 8 k,
      SCC): from the oracle's ground state, 30 leapfrog steps driven by the
      sin^2 pulse's values at its peak (steps 2067.. of the 20 fs pulse, A
      about 0.05 au from the first step), with the current (Eq. 14), energy,
      Tr(D S) and Mulliken charges of every step and two columns of both final
      levels (D_30, D_29) of every k-point.
  csi216_k216_kick20.npz - the 216-atom c-Si cell (864 orbitals) on the 6x6x6
      mesh (216 k), non-SCC: from the ground state, 20 steps after the kick
      A = 0.01 x, with J, E, Tr(D S) per step and sixteen seeded elements of
      both final levels of every k-point.

Run:  python tests/golden/make_fullsize_fixtures.py [asi512|csi216]
(about 10 and 15 minutes on 8 cores).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import vgtb_synth as vs  # noqa: E402

ASI512 = dict(name="asi512_k8_scc", start=2067, n_steps=30, cols=(5, 1234))
CSI216 = dict(name="csi216_k216", n_steps=20, n_samples=16, seed=216)


def asi512():
    c = vs.CONFIGS[ASI512["name"]]
    sysm = vs.config_system(ASI512["name"])
    full = vs.sin2_pulse_table(c["n_steps"], c["dt"], c["omega"], c["t_fs"] * vs.FS_AU, c["a_peak"])
    atab = full[ASI512["start"]:ASI512["start"] + ASI512["n_steps"]]
    t0 = time.time()
    d0, z, gap = oracle.ground_state(sysm)
    print(f"ground state {time.time() - t0:.0f} s, gap {gap:.3e}", flush=True)
    hist, st = oracle.propagate(sysm, d0, atab, c["dt"], ASI512["n_steps"], z=z)
    print(f"propagated {time.time() - t0:.0f} s", flush=True)
    cols = np.array(ASI512["cols"])
    out = dict(start=ASI512["start"], n_steps=ASI512["n_steps"], cols=cols, field=atab, z=z,
               J=hist["J"], E=hist["E"], trace=hist["trace"], q=hist["q"],
               cur_cols=np.stack([d[:, cols] for d in st.d_cur]),
               prev_cols=np.stack([d[:, cols] for d in st.d_prev]),
               cur_col_norm=np.array([np.linalg.norm(d[:, cols]) for d in st.d_cur]),
               gap=gap)
    np.savez(os.path.join(HERE, "asi512_k8_scc_pulse30.npz"), **out)


def csi216():
    c = vs.CONFIGS[CSI216["name"]]
    sysm = vs.config_system(CSI216["name"])
    n = sysm.n_orb
    rng = np.random.default_rng(CSI216["seed"])
    rows = rng.integers(0, n, size=(sysm.n_k, CSI216["n_samples"]))
    cols = rng.integers(0, n, size=(sysm.n_k, CSI216["n_samples"]))
    atab = vs.kick_table(1, c["a0"])
    t0 = time.time()
    d0, z, gap = oracle.ground_state(sysm)
    print(f"ground state {time.time() - t0:.0f} s, gap {gap:.3e}", flush=True)
    hist, st = oracle.propagate(sysm, d0, atab, c["dt"], CSI216["n_steps"], z=z)
    print(f"propagated {time.time() - t0:.0f} s", flush=True)
    kk = np.arange(sysm.n_k)[:, None]
    out = dict(n_steps=CSI216["n_steps"], rows=rows, cols=cols, J=hist["J"], E=hist["E"],
               trace=hist["trace"],
               cur=np.stack(st.d_cur)[kk, rows, cols], prev=np.stack(st.d_prev)[kk, rows, cols],
               d0_samples=np.stack(d0)[kk, rows, cols], gap=gap)
    np.savez(os.path.join(HERE, "csi216_k216_kick20.npz"), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["asi512", "csi216"]
    for w in which:
        {"asi512": asi512, "csi216": csi216}[w]()
