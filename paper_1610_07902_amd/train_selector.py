"""Train the schedule selector on the GPU from the library's own timings.

    python -m paper_1610_07902_amd.train_selector [--quick] [--out PATH]

Training graphs (the reading of the selector's training set): R-MAT scales
18, 20 and 22 (edge factor 16, symmetrised), a 2D 5-point grid 1024^2 and 3D
7-point grids 64^3, 128^3 and 192^3 (large enough that the pull direction's
cost per level, which grows with the unvisited vertices, is seen at the
sizes where it loses to push).  Samples: every BFS level from a few seeded
roots (min-select2nd, as a BFS step runs it: frontier expanded with the
visited vertices masked) plus standalone multiplies across densities for
plus-times and min-select2nd.  Each sample times all ten classes; the label
is the fastest.  Two networks of the same shape are trained by
spmspv_mlp_train_step, one on the BFS steps (for bfs_run) and one on the
standalone multiplies (for pagerank_run), and written as JSON next to this
file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import paper_1610_07902_amd as spv  # noqa: E402
from paper_1610_07902_amd import selector  # noqa: E402

DENSITIES = (1e-5, 1e-4, 3e-4, 1e-3, 3e-3, 1e-2, 3e-2, 1e-1, 3e-1)


def graphs(quick: bool):
    import synth
    if quick:
        yield "rmat14", synth.rmat(14, 16, seed=101, symmetrize=True)
        yield "rmat16", synth.rmat(16, 16, seed=102, symmetrize=True)
        yield "grid2d-256", synth.grid(256, 256, 1)
        yield "grid3d-32", synth.grid(32, 32, 32)
        return
    for s in (18, 20, 22):
        yield f"rmat{s}", synth.rmat(s, 16, seed=100 + s, symmetrize=True)
    yield "grid2d-1024", synth.grid(1024, 1024, 1)
    yield "grid3d-64", synth.grid(64, 64, 64)
    yield "grid3d-128", synth.grid(128, 128, 128)
    yield "grid3d-192", synth.grid(192, 192, 192)


def collect(quick: bool = False, roots_per_graph: int = 4, reps: int = 3, log=print) -> selector.Samples:
    import synth
    import torch
    out = selector.Samples()
    for name, A in graphs(quick):
        t0 = time.time()
        # pattern handle (BFS and min-select2nd) and a valued one (plus-times)
        P = spv.Matrix.from_csc(A, flags=spv.SYMMETRIC, pattern=True)
        # low-diameter graphs give few levels per root: take more roots
        roots = synth.roots(A, roots_per_graph * (3 if name.startswith("rmat") else 1), seed=7)
        s = selector.bfs_samples(P, A.nnz, roots, reps=reps, tag=name)
        s.extend(selector.random_samples(P, A.nnz, DENSITIES, spv.MIN_SELECT2ND_I32, reps=reps, seed=1,
                                         tag=name + "/min"))
        P.close()
        V = spv.Matrix.from_csc(A, flags=spv.WITH_TRANSPOSE)
        s.extend(selector.random_samples(V, A.nnz, DENSITIES, spv.PLUS_TIMES_F32, reps=reps, seed=2,
                                         tag=name + "/plus"))
        V.close()
        torch.cuda.empty_cache()
        out.extend(s)
        log(f"[train_selector] {name}: n={A.n} nnz={A.nnz} samples={len(s.raw)} ({time.time() - t0:.1f}s)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="small training graphs (tests)")
    ap.add_argument("--out", default=selector.WEIGHTS_PATH)
    ap.add_argument("--samples", default=None, help="also save the timing samples (.npz)")
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--roots", type=int, default=4)
    args = ap.parse_args()
    spv.load_library()
    t0 = time.time()
    samples = collect(args.quick, args.roots)
    if args.samples:
        samples.save(args.samples)
    # one network for BFS steps (with scale-augmented copies), one for
    # standalone multiplies
    bfs = samples.subset(samples.bfs_steps)
    mul = samples.subset(~samples.bfs_steps)
    params, mean, std, hist = selector.train(bfs, epochs=args.epochs)
    mp, mm, ms, mhist = selector.train(mul, epochs=args.epochs, scales=())
    import torch
    props = torch.cuda.get_device_properties(0)
    Tb, Tm = bfs.T, mul.T
    pb = selector.predict(params, mean, std, bfs.X)
    pm = selector.predict(mp, mm, ms, mul.X)
    meta = {"device": props.name, "arch": getattr(props, "gcnArchName", ""),
            "samples": len(samples.raw), "bfs_samples": len(bfs.raw), "multiply_samples": len(mul.raw),
            "epochs": args.epochs, "final_loss": hist[-1], "multiply_final_loss": mhist[-1],
            "train_accuracy": float((pb == Tb.argmin(1)).mean()),
            "train_regret": selector.regret(Tb, pb),
            "multiply_train_accuracy": float((pm == Tm.argmin(1)).mean()),
            "multiply_train_regret": selector.regret(Tm, pm),
            "label_histogram": np.bincount(Tb.argmin(1), minlength=10).tolist(),
            "multiply_label_histogram": np.bincount(Tm.argmin(1), minlength=10).tolist(),
            "seconds": round(time.time() - t0, 1), "quick": args.quick}
    selector.save_weights(params, mean, std, meta, args.out, multiply=(mp, mm, ms))
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
