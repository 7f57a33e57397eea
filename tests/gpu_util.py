"""Helpers shared by the GPU tests (no method arithmetic)."""
import sys

import numpy as np


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def per_field_rel_l2(a, b):
    return [rel_l2(a[c], b[c]) for c in range(a.shape[0])]
