"""Writes the oracle's reference traces for the two adaptive workloads.

Calls only the CPU oracle (``oracle/``) on inputs from the seeded generators
(``paper_1110_0573_amd.systems``); nothing here touches the GPU library.

  kerr_n60_t50.npz        driven damped Kerr cavity, N = 60, Dormand-Prince
                          rtol 1e-8, atol 1e-11, t in [0, 50], 101 outputs:
                          <a^+a>, <a> and the accepted / rejected step counts;
  tfim_8spin_t20_sample.npz
                          dissipative transverse-field Ising chain, 8 spins,
                          Dormand-Prince rtol 1e-7, atol 1e-10, t in [0, 20],
                          201 outputs, for a seeded sample of 4 of the 64
                          disorder realizations: all 8 <sigma_z^i> traces
                          and the step counts.

Run from the repository root:  python tests/golden/make_adaptive_golden.py
(about two minutes on 8 host cores).
"""
from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1110_0573_amd import systems as S  # noqa: E402

TFIM_SAMPLE_SEED = 2024
TFIM_SAMPLE = 4


def tfim_sample_indices(n_inst=64):
    """The realizations whose oracle traces are stored (seeded, without replacement)."""
    rng = np.random.default_rng(TFIM_SAMPLE_SEED)
    return np.sort(rng.choice(n_inst, TFIM_SAMPLE, replace=False))


def main():
    kw = S.kerr_single()
    tw = S.tfim()
    idx = tfim_sample_indices(len(tw.systems))
    jobs = [("kerr", kw.systems[0], kw)] + [("tfim", tw.systems[i], tw) for i in idx]

    def run(job):
        _, s, w = job
        t0 = time.perf_counter()
        r = oracle.dopri5(s, s.rho0, w.tlist, w.rtol, w.atol)
        return r, time.perf_counter() - t0

    with ThreadPoolExecutor(len(jobs)) as ex:
        res = list(ex.map(run, jobs))
    (rk, tk) = res[0]
    np.savez(os.path.join(HERE, "kerr_n60_t50.npz"), tlist=kw.tlist, expect=rk["expect"],
             counts=rk["counts"], rtol=kw.rtol, atol=kw.atol)
    print(f"kerr: {rk['counts'][0]} accepted, {rk['counts'][1]} rejected, {tk:.1f} s")
    ex_t = np.stack([r["expect"] for r, _ in res[1:]])
    counts = np.stack([r["counts"] for r, _ in res[1:]])
    np.savez(os.path.join(HERE, "tfim_8spin_t20_sample.npz"), tlist=tw.tlist, index=idx,
             expect=ex_t, counts=counts, rtol=tw.rtol, atol=tw.atol)
    for i, (r, t) in zip(idx, res[1:]):
        print(f"tfim[{i}]: {r['counts'][0]} accepted, {r['counts'][1]} rejected, {t:.1f} s")


if __name__ == "__main__":
    main()
