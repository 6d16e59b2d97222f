"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def say(*a):
    """Print and flush: names the case before a GPU step runs."""
    print(*a, flush=True)
    sys.stdout.flush()


def rel(y, ref):
    """Normwise relative error max|y - y*| / max|y*| over a component group."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(y - ref))) if ref.size else 0.0
    return num / den if den > 0 else num


def group_errors(gpu: dict, ref: dict) -> dict:
    return {k: rel(gpu[k], ref[k]) for k in ref if gpu.get(k) is not None}


ELEM_FLOOR = 1e-3


def elem_rel(y, ref) -> np.ndarray:
    """Elementwise relative error |y - y*| / (|y*| + 1e-3 max|y*|) of every
    element of a component group (the floor keeps elements near a node of
    the orbital from dividing by ~0)."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    if ref.size == 0:
        return np.zeros(0)
    den = np.abs(ref) + ELEM_FLOOR * float(np.max(np.abs(ref)))
    den = np.where(den > 0, den, 1.0)
    return np.abs(y - ref) / den


def error_report(gpu: dict, ref: dict) -> dict:
    """Per component group: the normwise error, and the 99th percentile and
    maximum of the elementwise error."""
    out = {}
    for k in ref:
        if gpu.get(k) is None:
            continue
        e = elem_rel(gpu[k], ref[k])
        out[k] = {"norm": rel(gpu[k], ref[k]),
                  "elem_p99": float(np.percentile(e, 99)) if e.size else 0.0,
                  "elem_max": float(np.max(e)) if e.size else 0.0}
    return out


def format_report(rep: dict) -> str:
    return " ".join(f"{k}: norm {v['norm']:.2e} p99 {v['elem_p99']:.2e} max {v['elem_max']:.2e}"
                    for k, v in rep.items())


def to_np(t):
    return None if t is None else t.detach().cpu().numpy()


def quantize_bf16(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even FP32 -> BF16 -> FP32 (via torch's CPU cast)."""
    import torch
    f = np.ascontiguousarray(x).view(np.float32)
    q = torch.from_numpy(f).to(torch.bfloat16).to(torch.float32).numpy()
    return q.view(x.dtype).reshape(x.shape)


def quantize_f16_scaled(x: np.ndarray) -> np.ndarray:
    """The documented FP16 storage rule: a * 2^e rounded to half (RNE), with
    e putting max|a| into (2^13, 2^14]; returned divided by 2^e."""
    f = np.ascontiguousarray(x).view(np.float32)
    mx = float(np.max(np.abs(f[np.isfinite(f)]))) if f.size else 0.0
    e = 0 if mx == 0.0 else int(max(-24, min(24, 14 - int(np.ceil(np.log2(mx))))))
    q = (f * np.float32(2.0 ** e)).astype(np.float16).astype(np.float32) * np.float32(2.0 ** -e)
    return q.view(x.dtype).reshape(x.shape)
