"""Writes fullsize_<scene>_100.npz: the FP64 oracle's state after 100
substeps of the full c2 (1,048,576 particles, 128^3) and c3 (4,194,304
particles, 256^3) scenes, on a seeded sample of particles.

Algorithm 1 (Sec. III-B) with the grid contact of Sec. IV-A, run by the
oracle alone on the whole scene (no cone-of-influence cut: after 100
substeps a particle depends on the whole slab). The sample is 2,000
particles drawn uniformly plus 1,000 from boxes around each tool's path,
where contact decides the result. Stored per sampled particle: its index
and the oracle's x, v, C, F; per scene: the tool impulses of the 100
substeps, the oracle's status and a SHA-256 of the generated inputs (the
test refuses a golden whose inputs no longer match the generator).

Run from the repository root: python tests/golden/make_fullsize.py [c2] [c3]
(about 1 minute for c2 and 3-4 minutes for c3 on one core).
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2502_18437_amd import scenes  # noqa: E402  (input generator only)
from tests.parity import run_oracle  # noqa: E402  (calls oracle/ only)

N_SUBSTEPS = 100
N_UNIFORM = 2000
N_PER_TOOL = 1000


def input_digest(s):
    h = hashlib.sha256()
    for a in (s.x, s.E):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    for t in s.tools:
        h.update(repr(t.kwargs()).encode())
    h.update(repr((s.n_grid, s.dt, s.nu, s.E_default, s.mass, s.vol0)).encode())
    return h.hexdigest()


def sample(s, seed):
    rng = np.random.default_rng(seed)
    picks = [rng.choice(s.N, N_UNIFORM, replace=False)]
    for t in s.tools:
        # particles within a few cells of the tool's centre line over the run
        c0 = np.asarray(t.center)
        c1 = c0 + N_SUBSTEPS * s.dt * np.asarray(t.lin_vel)
        reach = max(t.size) + 4 * s.dx
        lo, hi = np.minimum(c0, c1) - reach, np.maximum(c0, c1) + reach
        near = np.nonzero(np.all((s.x >= lo) & (s.x <= hi), axis=1))[0]
        if near.size:
            picks.append(rng.choice(near, min(N_PER_TOOL, near.size), replace=False))
    return np.unique(np.concatenate(picks)).astype(np.int64)


def make(name):
    s = scenes.make(name)
    idx = sample(s, seed=100 + s.n_grid)
    t0 = time.perf_counter()
    o = run_oracle(s, N_SUBSTEPS)
    dt = time.perf_counter() - t0
    out = os.path.join(HERE, f"fullsize_{name}_{N_SUBSTEPS}.npz")
    np.savez_compressed(out, idx=idx, x=o["x"][idx], v=o["v"][idx], C=o["C"][idx], F=o["F"][idx],
                        impulses=o["impulses"], status=np.int64(o["status"]),
                        n_substeps=np.int64(N_SUBSTEPS), input_sha256=np.array(input_digest(s)),
                        oracle_seconds=np.float64(dt))
    print(f"{name}: {s.N} particles, {N_SUBSTEPS} substeps in {dt:.1f} s, {idx.size} sampled -> {out}",
          flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["c2", "c3"]):
        make(name)
