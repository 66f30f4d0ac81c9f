"""Shared helpers of the GPU parity tests (inputs, oracle calls, error norms)."""

import math
import sys

import numpy as np

import synth

SIGMA_SKY = math.sqrt(synth.SKY_LEVEL)
TOL_FP32 = 1e-4 * SIGMA_SKY      # max |dD| for the FP32 path
TOL_MFMA = 1e-2 * SIGMA_SKY      # max |dD| for the bf16 / fp16 forms


def say(*args):
    """Name the case before each GPU step (flushed, so a fault still shows it)."""
    print(*args, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def err_stats(got, want, mask=None):
    d = np.abs(np.asarray(got, np.float64) - np.asarray(want, np.float64))
    if mask is not None:
        d = d[mask]
    return float(d.max()), float(np.sqrt(np.mean(d * d)))


def sample_pixels(H, W, n, seed, R=None, h=0):
    """n random pixels, every corner and edge band pixel class, and (if R is
    given) the 32 brightest pixels of R."""
    r = np.random.default_rng(seed)
    xs = list(r.integers(0, W, n))
    ys = list(r.integers(0, H, n))
    for y in (0, 1, h, H // 2, H - 1 - h, H - 2, H - 1):
        for x in (0, 1, h, W // 2, W - 1 - h, W - 2, W - 1):
            if 0 <= x < W and 0 <= y < H:
                xs.append(x)
                ys.append(y)
    if R is not None:
        flat = np.argsort(R.ravel())[-32:]
        ys += list(flat // W)
        xs += list(flat % W)
    return np.array(xs, dtype=np.int32), np.array(ys, dtype=np.int32)


_INPUTS = {}


def workload_images(name):
    """(R, a, I) of a workload (synth recipe), generated once per test session."""
    if name not in _INPUTS:
        wl = synth.WORKLOADS[name]
        R, a = synth.workload_inputs(wl)
        _INPUTS[name] = (R, a, synth.second_image(wl))
    return _INPUTS[name]
