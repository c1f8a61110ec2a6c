"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np


def say(*a):
    """Name the case before each GPU step, flushed, so a crash log shows it."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def field_parity(gpu, ref, tol_rel, floor_frac=1e-6):
    """Per-variable relative L2 and infinity-norm errors of a [5][E][n] field.
    A variable whose reference norm is below floor_frac of the largest one is
    measured against that floor instead (its own norm is only discretisation
    noise)."""
    gpu = np.asarray(gpu, dtype=np.float64).reshape(5, -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(5, -1)
    norms = np.linalg.norm(ref, axis=1)
    infs = np.max(np.abs(ref), axis=1)
    floor = floor_frac * norms.max()
    l2 = [np.linalg.norm(gpu[v] - ref[v]) / max(norms[v], floor) for v in range(5)]
    li = [np.max(np.abs(gpu[v] - ref[v])) / max(infs[v], floor_frac * infs.max()) for v in range(5)]
    return np.array(l2), np.array(li)


def periodic_patch(blocks, centre, radius):
    """Sub-block of a [5, N, N, N, k, j, i] array around element (ez, ey, ex),
    radius elements each way, wrapping periodically."""
    N = blocks.shape[1]
    idx = [np.arange(c - radius, c + radius + 1) % N for c in centre]
    return blocks[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]


def state_parity(gpu, ref):
    """Per-variable relative L2 and infinity-norm errors of a state [5][E][n]
    in which the three momentum components share one scale (the momentum
    vector's norm): a component that starts at zero and holds only what the
    others feed into it (rho w of the Taylor-Green vortex) is measured against
    the flow's momentum, not against its own small size."""
    gpu = np.asarray(gpu, dtype=np.float64).reshape(5, -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(5, -1)
    norms = np.linalg.norm(ref, axis=1)
    infs = np.max(np.abs(ref), axis=1)
    norms[1:4] = np.linalg.norm(ref[1:4])
    infs[1:4] = np.max(np.abs(ref[1:4]))
    l2 = np.linalg.norm(gpu - ref, axis=1) / norms
    li = np.max(np.abs(gpu - ref), axis=1) / infs
    return l2, li
