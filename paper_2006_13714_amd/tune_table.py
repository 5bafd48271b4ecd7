"""Regenerate the packaged autotuner table (tuned_gfx950.txt) on an MI355X.

Usage: python -m paper_2006_13714_amd.tune_table OUT_FILE [--reps N] [--append-slabs]
       [--append-paper]

Runs bm_autotune for the shape classes of the library's workloads -- grayscale and colour
images with 6x6 / 8x8 patches at stride 3 in a 39x39 window (K = 16), 2..4-channel 8x8
patches, and 4-channel 8x8 patches at stride 4 in a 31x31 window (K = 32) -- in every
precision form, over the three reference-grid size buckets per axis, plus the one-slab
problems of the 3D search workloads (256 x 256, 6 x 6 patches, stride 1, 30 x 30 window,
1 or 3 planes), plus the paper's single-channel runtime setup (6 x 6 patches, stride 1,
30 x 30 window, K = 16) on 512- and 1024-pixel sides -- each timed on a synthetic image of
that class, and writes one "<class> | <configuration>" line per class.  --append-slabs
(--append-paper) tunes only the slab (paper-setup) classes and appends them to an existing
table.
"""
from __future__ import annotations

import argparse
import os
import sys


def slab_classes():
    """The one-slab 2D problems of the 3D search workloads (256 x 256 planes, 6 x 6 patches,
    stride 1, 30 x 30 windows, K = 16; 1-plane and 3-plane blocks): 3D plans look these up."""
    return [(256, 256, C, 6, 1, 30, 16, prec) for prec in ("fp32", "bf16x4", "fp16x3")
            for C in (1, 3)]


def paper_classes():
    """The paper's single-channel runtime setup (Sec. V-A: 6 x 6 patches, stride 1, 30 x 30
    window), K = 16, on 512 x 512 and 1024 x 1024 images, in every form."""
    return [(side, side, 1, 6, 1, 30, 16, prec) for prec in ("fp32", "bf16x4", "fp16x3")
            for side in (512, 1024)]


def classes():
    sides = (128, 512, 1024)  # one per reference-grid size bucket
    out = []
    for prec in ("fp32", "bf16x4", "fp16x3"):
        for C in (1, 2, 3, 4):
            for P in ((6, 8) if C in (1, 3) else (8,)):
                for H in sides:
                    for W in sides:
                        out.append((H, W, C, P, 3, 39, 16, prec))
        out.append((1024, 1024, 4, 8, 4, 31, 32, prec))
    return out + slab_classes() + paper_classes()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--reps", type=int, default=8)
    ap.add_argument("--append-slabs", action="store_true",
                    help="only tune the 3D workloads' slab classes, appending to OUT_FILE")
    ap.add_argument("--append-paper", action="store_true",
                    help="only tune the paper-setup classes, appending to OUT_FILE")
    a = ap.parse_args()
    out = os.path.abspath(a.out)
    if not (a.append_slabs or a.append_paper):
        with open(out, "w") as f:
            f.write("# autotuner table for gfx950 (MI355X), written by "
                    "paper_2006_13714_amd.tune_table\n# <shape class> | <kernel configuration>\n")
    # bm_autotune appends each class's winner to this file under the library's own key
    os.environ["BM_TUNE_CACHE"] = out
    os.environ.pop("BM_CFG", None)
    import torch
    from paper_2006_13714_amd import bm, synth
    todo = (slab_classes() if a.append_slabs else paper_classes() if a.append_paper
            else classes())
    for (H, W, C, P, s, Wn, K, prec) in todo:
        img = (synth.gray_voronoi(7, H, W, 50.0) if C == 1 else
               synth.multichannel_voronoi(7, H, W, C, 50.0, nir=(C == 4)))
        t = torch.from_numpy(img).cuda()
        cfg = bm.bm_autotune(bm.make_desc(H, W, C, P, s, Wn, K, prec), t, a.reps)
        print(f"{H}x{W}x{C} P{P} s{s} w{Wn} K{K} {prec}: {cfg}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
