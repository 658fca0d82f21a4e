"""Writes tests/golden/full_solve_512x512x64_40views.npz: the FP64 oracle's Algorithm A1 with the
two-level cascade of Section II.C.3 ([20, 20] outer iterations, lambda = 0.05, Schur step per
level) on the 512 x 512 x 64 / 40-view / 512 x 384 workload, seeded ellipsoid phantom 21 and
Poisson noise 22 at I0 = 1e5.

Calls only the oracle and the input generators.  The stored arrays:
  y_sha256       digest of the float64 projections the oracle solved (the GPU test regenerates
                 them from the seeds and checks the digest before comparing anything)
  trace, rof_e   the ROF decision trace (level, outer, inner, m) and E_0, E_trial, G per record
  energy, t_used E(f_k) per outer iteration (coarsest level first) and t per level
  vox, f_vox     20000 seeded voxel indices (flat, [nz][ny][nx]) and the final volume there
  f_norm         the final volume's L2 norm (the relative error bar's denominator)
  seconds, threads  oracle wall time and OpenMP threads of this run (reported, not compared)

Run from the repository root:  python tests/golden/make_full_solve_golden.py [threads]
(about 20 minutes on 8 cores)."""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cbct_synth as S  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "full_solve_512x512x64_40views.npz")
N_SAMPLES = 20000
SAMPLE_SEED = 23


def inputs():
    """The workload's projections (float64), from the seeds alone."""
    cfg = S.CONFIGS["wide512x512x64"]
    g = cfg["geometry"]
    ph = S.make_phantom(g, cfg["seeds"][0])
    Y = S.poisson_log(S.analytic_projections(g, ph), cfg["I0"], cfg["seeds"][1])
    return g, cfg, np.ascontiguousarray(Y, dtype=np.float64)


def digest(Y):
    return hashlib.sha256(np.ascontiguousarray(Y, dtype=np.float64).tobytes()).hexdigest()


def sample_voxels(g):
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(g.n_vox, size=N_SAMPLES, replace=False)).astype(np.int64)


def main():
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    g, cfg, Y = inputs()
    t0 = time.time()
    res = oracle.reconstruct(g, Y, cfg["lam"], cfg["iters"], cfg["levels"])
    secs = time.time() - t0
    vox = sample_voxels(g)
    f = res.f.ravel()
    np.savez_compressed(OUT, y_sha256=np.array(digest(Y)), trace=res.trace.astype(np.int32), rof_e=res.rof_e,
                        energy=res.energy, t_used=np.array(res.t_used), vox=vox, f_vox=f[vox],
                        f_norm=np.array(np.linalg.norm(f)), seconds=np.array(secs),
                        threads=np.array(oracle.get_threads()), iters=np.array(cfg["iters"]),
                        lam=np.array(cfg["lam"]))
    print("oracle [20, 20] solve: %.1f s on %d threads, %d ROF records; wrote %s"
          % (secs, oracle.get_threads(), len(res.trace), OUT), flush=True)


if __name__ == "__main__":
    main()
