"""Write the stored oracle values of the full-size workloads.

Every number this script writes comes from the FP64 CPU oracle (``oracle/``)
on inputs from ``paper_2105_08806_amd.inputs``; nothing comes from the GPU
library.  It is run once, on the CPU; the GPU parity tests read the files.

    python tests/golden/make_golden.py c2     # 2D N=64 VHS, all 4096 coefficients
    python tests/golden/make_golden.py c3     # 3D N=32 BKW, 256 coefficients, all 64 directions
    python tests/golden/make_golden.py a3     # 3D N=32, angle-dependent rate, one direction pair

c2: the 2D variable-hard-sphere workload (64 modes, S = 6, B = |u|/(2 pi),
    32 circle directions, two Maxwellians of mass 1/2 at +-(1.5, 0) with
    seeded temperatures).  Q and Q+ of every coefficient for the FP64 input
    and for the same input rounded to FP32 (the FP32 plan's input).
c3: the 3D BKW workload (32 modes, S = 5, Maxwell B = 1/(4 pi), BKW data at
    t = 6.5, the 8 x 8 product rule).  The gain is linear in the direction
    rule, so it is summed per antipodal pair of directions (32 pairs) and
    written pair by pair; the full-rule Q+ is the sum over pairs, and any
    union of pairs is a valid smaller rule.  Q- is written per pair as well.
    256 coefficients: the product set {0, 1, 4, 15, 30, 31}^3 (edges, odd and
    even indices) and 40 seeded random multi-indices.
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2105_08806_amd import inputs as I  # noqa: E402

C2_FILE = os.path.join(HERE, "c2_vhs2d_n64.txt")
C3_FILE = os.path.join(HERE, "c3_bkw3d_n32_pairs.txt")
A3_FILE = os.path.join(HERE, "a3_aniso3d_n32_pair.txt")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()[:16]


def c2_problem():
    N, S, M = 64, 6.0, 32
    sg, sw = O.circle_rule(M)
    ora = O.Problem(2, N, S, 0, kernel="vhs", b0=1.0 / (2 * np.pi), gamma=1.0, sphere=sg, sphere_w=sw)
    c = ora.project(I.mixture(ora.interior_velocities(), I.two_maxwellians_2d()))
    return ora, c


def c3_setup():
    N, S = 32, 5.0
    sg, sw = O.sphere_product_rule(8, 8)
    pairs, seen = [], set()
    for a in range(len(sw)):
        if a in seen:
            continue
        b = int(np.argmin(np.linalg.norm(sg + sg[a], axis=1)))
        seen.update((a, b))
        pairs.append((a, b))
    full = O.Problem(3, N, S, 0, sphere=sg, sphere_w=sw)
    c = full.project(I.bkw_f(6.5, full.interior_velocities()))
    pick = [0, 1, 4, 15, 30, 31]
    grid = np.stack(np.meshgrid(*([pick] * 3), indexing="ij"), -1).reshape(-1, 3)
    rnd = np.random.default_rng(3232).integers(0, N, size=(40, 3))
    kidx = np.concatenate([grid, rnd]).astype(np.int32)
    return sg, sw, pairs, c, kidx


def make_c2():
    ora, c = c2_problem()
    c32 = c.astype(np.float32).astype(np.float64)
    cols = []
    for cin in (c, c32):
        t = time.time()
        q, qp, _ = ora.collision(cin)
        print("c2: one full evaluation in %.0f s" % (time.time() - t), flush=True)
        cols += [q.ravel(), qp.ravel()]
    with open(C2_FILE, "w") as f:
        f.write("# 2D VHS workload, N=64, S=6, B=|u|/(2 pi), 32 directions, two Maxwellians (seed 2105)\n")
        f.write("# written by tests/golden/make_golden.py c2 from the FP64 CPU oracle (oracle/)\n")
        f.write("# input sha256[:16] fp64 %s fp32-rounded %s\n" % (digest(c), digest(c32)))
        f.write("# k1 k2 Q Q+ (FP64 input) Q Q+ (input rounded to FP32)\n")
        N = c.shape[0]
        for r in range(N * N):
            f.write("%d %d %s\n" % (r // N, r % N, " ".join("%.17e" % col[r] for col in cols)))


def make_c3():
    sg, sw, pairs, c, kidx = c3_setup()
    done = set()
    if os.path.exists(C3_FILE):
        for line in open(C3_FILE):
            if line.startswith("pair "):
                done.add(int(line.split()[1]))
    else:
        with open(C3_FILE, "w") as f:
            f.write("# 3D BKW workload, N=32, S=5, Maxwell B=1/(4 pi), t0=6.5, 8x8 product rule\n")
            f.write("# written by tests/golden/make_golden.py c3 from the FP64 CPU oracle (oracle/)\n")
            f.write("# input sha256[:16] %s\n" % digest(c))
            f.write("kidx %s\n" % " ".join("%d,%d,%d" % tuple(k) for k in kidx))
    for p, (a, b) in enumerate(pairs):
        if p in done:
            continue
        ora = O.Problem(3, 32, 5.0, 0, sphere=sg[[a, b]], sphere_w=sw[[a, b]])
        t = time.time()
        qp, qm = ora.collision_at(c, kidx)
        print("c3: pair %d (%d, %d) in %.0f s" % (p, a, b, time.time() - t), flush=True)
        with open(C3_FILE, "a") as f:
            f.write("pair %d %d %d\n" % (p, a, b))
            f.write("qplus %s\n" % " ".join("%.17e" % x for x in qp))
            f.write("qminus %s\n" % " ".join("%.17e" % x for x in qm))


def a3_setup():
    """3D, 32 modes, S = 5, the angle-dependent rate B = b0 |u| (1 + 2 cos^2 theta),
    one antipodal pair of the 8 x 8 product rule off the axes (direction 13 and
    its antipode), a two-Maxwellian input; 22 multi-indices."""
    N, S = 32, 5.0
    sg, sw = O.sphere_product_rule(8, 8)
    s0 = 13
    s1 = int(np.argmin(np.linalg.norm(sg + sg[s0], axis=1)))
    ora = O.Problem(3, N, S, 0, kernel="aniso", aniso=2.0, gamma=1.0, sphere=sg[[s0, s1]], sphere_w=sw[[s0, s1]])
    comps = [(0.6, (0.5, -0.3, 0.1), 0.7), (0.4, (-0.8, 0.6, 0.2), 1.2)]
    c = ora.project(I.mixture(ora.interior_velocities(), comps))
    rnd = np.random.default_rng(3233).integers(0, N, size=(20, 3))
    kidx = np.concatenate([[[0, 0, 0], [N - 1, N - 1, N - 1]], rnd]).astype(np.int32)
    return ora, c, kidx, (s0, s1)


def make_a3():
    ora, c, kidx, (s0, s1) = a3_setup()
    t = time.time()
    qp, qm = ora.collision_at(c, kidx)
    print("a3: %d coefficients in %.0f s" % (len(kidx), time.time() - t), flush=True)
    with open(A3_FILE, "w") as f:
        f.write("# 3D N=32, S=5, B = b0 |u| (1 + 2 cos^2 theta), directions %d and %d of the 8x8 product rule, "
                "two Maxwellians\n" % (s0, s1))
        f.write("# written by tests/golden/make_golden.py a3 from the FP64 CPU oracle (oracle/)\n")
        f.write("# input sha256[:16] %s\n" % digest(c))
        f.write("kidx %s\n" % " ".join("%d,%d,%d" % tuple(k) for k in kidx))
        f.write("qplus %s\n" % " ".join("%.17e" % x for x in qp))
        f.write("qminus %s\n" % " ".join("%.17e" % x for x in qm))


if __name__ == "__main__":
    for what in sys.argv[1:] or ["c2", "c3", "a3"]:
        {"c2": make_c2, "c3": make_c3, "a3": make_a3}[what]()
