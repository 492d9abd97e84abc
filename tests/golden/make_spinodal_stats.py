"""Writes spinodal256_stats.txt: late-time statistics of the spinodal workload (1024^2 workload
parameters on a 256^2 periodic grid) from the FP64 oracle alone.

For each variant (QIM, IM) and seed (0, 1, 2) the oracle starts from the seeded field
phi = 0.5 + U[-0.005, 0.005] rounded to FP32 (what the GPU receives) and steps to t = 20000;
at t = 2000, 5000, 10000 and 20000 it records sum(phi) and the characteristic length of
oracle.stats. Runs the six trajectories in parallel processes (about 10 minutes).

python tests/golden/make_spinodal_stats.py
"""
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N = 256
TIMES = (2000, 5000, 10000, 20000)
OUT = os.path.join(HERE, "spinodal256_stats.txt")


def run(args):
    import numpy as np

    import oracle
    from oracle import stats
    from paper_1902_08933_amd import workloads as W
    variant, seed = args
    cfg, phi = W.spinodal(n=N, variant=variant, seed=seed)
    o = oracle.Oracle(cfg).init(phi.astype(np.float32).astype(np.float64))
    rows, t = [], 0
    for t_next in TIMES:
        o.step(t_next - t)
        t = t_next
        rows.append((variant, seed, t, o.sum_phi(), stats.characteristic_length(o.read("phi"))))
    return rows


def main():
    jobs = [(v, s) for v in ("qim", "im") for s in (0, 1, 2)]
    with Pool(len(jobs)) as pool:
        res = pool.map(run, jobs)
    with open(OUT, "w") as fh:
        fh.write("# Spinodal decomposition, 256 x 256 periodic, parameters of the 1024^2 workload\n"
                 "# (rho ratio 3, nu_A = 0.1, nu_B = 1, sigma 0.03, W 4, M_phi 0.1, tau_h 1,\n"
                 "# F_s = mu grad phi, eq. (28)), phi0 = 0.5 + U[-0.005, 0.005] (numpy PCG64 seed),\n"
                 "# rounded to FP32. FP64 oracle; written by tests/golden/make_spinodal_stats.py.\n"
                 "# columns: variant seed step sum_phi characteristic_length\n")
        for rows in res:
            for v, s, t, sp, L in rows:
                fh.write(f"{v} {s} {t} {sp:.17g} {L:.10g}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
