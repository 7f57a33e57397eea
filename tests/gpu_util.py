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


def sparse_modes(K, count, seed, edge=4):
    """Random real solenoidal velocity with `count` modes (plus conjugate
    partners) in |k_j| <= K, `edge` of them on the band's faces |k_j| = K, as a
    {(kx, ky, kz): u_hat} dict (test input)."""
    rng = np.random.default_rng(seed)
    modes = {}
    while len(modes) < 2 * count:
        k = [int(x) for x in rng.integers(-K, K + 1, size=3)]
        if len(modes) < 2 * edge:
            k[int(rng.integers(0, 3))] = K * (1 if rng.random() < 0.5 else -1)
        k = tuple(k)
        if k == (0, 0, 0) or k in modes:
            continue
        kv = np.array(k, dtype=float)
        a = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        a = (a - kv * (kv @ a) / (kv @ kv)) * 0.01
        modes[k] = a
        modes[(-k[0], -k[1], -k[2])] = np.conj(a)
    return modes


def modes_to_half_spectrum(modes, n):
    uh = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    for k, a in modes.items():
        if k[0] >= 0:
            uh[:, k[2] % n, k[1] % n, k[0]] = a
    return uh


def compare_with_modes(got, expect, n, rel):
    """max |got - f| over every entry (f from the mode dict, zero elsewhere)
    relative to max |f|."""
    scale = max(float(np.abs(f).max()) for f in expect.values())
    ref_at = np.zeros_like(got)
    for k, f in expect.items():
        ref_at[:, k[2] % n, k[1] % n, k[0]] = f
    err = float(np.abs(got - ref_at).max()) / scale
    assert err <= rel, err
    return err
