"""Shared helpers for the parity tests (no arithmetic of the method here)."""
import functools
import time

import numpy as np

import oracle
from oracle import geometry as og
from oracle import phantom as oph
import workloads as wl


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def log(*args):
    print("[%s]" % time.strftime("%H:%M:%S"), *args, flush=True)


@functools.lru_cache(maxsize=4)
def c1_filtered(index: int = 0):
    """Ramp-filtered analytic projections of C1 phantom ``index`` (oracle side):
    float32 [64, 128, 128] and the world matrices."""
    cfg = wl.CONFIGS["c1"]
    ell = wl.config_ellipsoids(cfg, index)
    raw = oph.line_integrals(ell, cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    filt = oracle.fdk_filter(raw, cfg["scan"]).astype(np.float32)
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    return filt, mats
