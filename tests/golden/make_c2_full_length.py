"""Writes tests/golden/c2_full_length_oracle.json: the CPU oracle's results
for two trajectories of each of the four (kappa_hat, gamma_hat) runs of the
N = 2048 Bjorken batch (4096 trajectories, 11,899 steps, Gaussian l = 0
singlet of width 0.2 fm; see paper_2107_06147_amd.workloads.c2_headline),
over the whole run.  Calls only the oracle.  About a minute per trajectory
and core:

    python tests/golden/make_c2_full_length.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2107_06147_amd import workloads as W  # noqa: E402

IDS = (0, 2047)
OUT = os.path.join(HERE, "c2_full_length_oracle.json")


def one(job):
    kh, gh, tid = job
    r = oracle.run(W.c2_headline(kh, gh), n_traj=1, traj_id0=tid, jump_log_cap=64, n_threads=1)
    n = int(r["n_jumps"][0])
    row = {
        "kappa_hat": kh, "gamma_hat": gh, "traj_id": tid, "n_steps": int(r["n_steps"]),
        "status": int(r["status"][0]), "steps_done": int(r["steps_done"][0]),
        "n_jumps": n, "l": int(r["l"][0]), "color": int(r["color"][0]),
        "norm": float(r["norm"][0]), "first_r": float(r["first_r"][0]),
        "min_gap": float(r["min_gap"][0]), "mean_r": float(r["mean_r"][0]),
        "overlap": [float(x) for x in r["overlap"][0]],
        "survival": [float(x) for x in r["survival"][0]],
        "jump_log": [[int(e[0]), int(e[1]), int(e[2])] for e in r["jump_log"][0][:min(n, 64)]],
    }
    print(kh, gh, tid, n, row["norm"], flush=True)
    return row


def main():
    from multiprocessing import Pool
    jobs = [(kh, gh, tid) for (kh, gh) in W.C2_RUNS for tid in IDS]
    with Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        rows = pool.map(one, jobs)
    json.dump({"source": "oracle/qtraj_oracle.c via tests/golden/make_c2_full_length.py",
               "rows": rows}, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
