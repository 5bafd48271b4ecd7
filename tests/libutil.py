"""Shared test helpers: locate/build the library, GPU tensors, case banners."""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    from paper_2006_13714_amd import bm
    if not os.path.exists(bm.LIB_PATH):
        from paper_2006_13714_amd import build_lib
        build_lib.build()
    return bm


def banner(msg: str):
    """Name the case on stdout before it touches the GPU (survives a lost box)."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()
