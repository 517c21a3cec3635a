"""Write the expected fields of the long FP32 parity runs (tests/test_gpu_longrun.py).

    python tests/golden/make_longrun.py [ternary_2d] [quaternary_3d]

Each case runs the FP64 oracle (``oracle.lbm``) for the full number of steps of
its workload on a smaller lattice, with the inputs of ``workloads`` (seeded
generators that hold none of the method), and stores the observables at a
fixed sample of nodes together with whole-field diagnostics:

* ``ternary_2d``:    1024^2 D2Q5 ternary, the field generator and D_ij of the
                     4096^2 workload (seed 1), periodic, 2000 steps;
* ``quaternary_3d``: 64^3 D3Q7 quaternary, the two-slab field and D_ij of the
                     512^3 workload (seed 2), zero-flux x walls, periodic y and
                     z, 500 steps.

Nothing here calls the HIP library.  Output: ``longrun_<case>.npz`` next to
this script (numpy arrays only, no pickles).  The 2D case takes ten to thirty
minutes on one core.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import lbm  # noqa: E402
import workloads  # noqa: E402

SAMPLE_SEED = 20240611
SAMPLES = 2048


def case_workload(name):
    if name == "ternary_2d":
        return workloads.ternary_2d(shape=(1024, 1024), seed=1, steps=2000)
    if name == "quaternary_3d":
        return workloads.quaternary_3d(shape=(64, 64, 64), seed=2, steps=500)
    raise SystemExit(f"unknown case {name}")


def sample_nodes(shape):
    """Flat node indices (x fastest): SAMPLES distinct random nodes, plus every node
    of two lines along each axis, one through the centre and one through the
    corner at the origin (faces and wrap-around neighbours included)."""
    rng = np.random.default_rng(SAMPLE_SEED)
    nodes = int(np.prod(shape))
    pick = set(rng.choice(nodes, size=min(SAMPLES, nodes), replace=False).tolist())
    strides = np.cumprod((1,) + tuple(shape[:-1]))
    mid = [n // 2 for n in shape]
    for a, n in enumerate(shape):
        for fixed in (mid, [0] * len(shape)):
            for j in range(n):
                c = list(fixed)
                c[a] = j
                pick.add(int(sum(ci * st for ci, st in zip(c, strides))))
    return np.array(sorted(pick), dtype=np.int64)


def make(name):
    w = case_workload(name)
    prob = lbm.Problem(w.lattice, w.D, w.shape, bc=w.bc)
    t0 = time.perf_counter()
    f = lbm.run(prob, w.xi0, w.steps)
    xi, grad, J = lbm.observables(prob, f)
    totals, mins, maxs, nonfinite = lbm.diagnostics(prob, f)
    idx = sample_nodes(w.shape)
    flat = lambda a: a.reshape(a.shape[: a.ndim - len(w.shape)] + (-1,))[..., idx]
    out = os.path.join(HERE, f"longrun_{name}.npz")
    np.savez_compressed(
        out,
        shape=np.array(w.shape, dtype=np.int64),
        steps=np.array(w.steps, dtype=np.int64),
        D=w.D,
        idx=idx,
        xi=flat(xi),
        J=flat(J),
        grad=flat(grad),
        totals=totals,
        xi0_totals=w.xi0.reshape(w.N, -1).sum(axis=1),
        mins=mins,
        maxs=maxs,
        nonfinite=np.array(nonfinite, dtype=np.int64),
    )
    print(f"{name}: {w.lattice} {w.shape} x {w.steps} steps in {time.perf_counter() - t0:.0f} s -> {out} "
          f"({idx.size} sampled nodes)", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["ternary_2d", "quaternary_3d"]:
        make(name)
