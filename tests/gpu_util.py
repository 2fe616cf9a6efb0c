"""Helpers for the GPU parity tests: move seeded inputs to the device through
the binding, and compare against the FP64 oracle."""
import numpy as np
import torch

from paper_1406_4519_amd import dfacto, gen

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def coo_to_dev(coo):
    i = torch.from_numpy(np.ascontiguousarray(coo.i).view(np.int32)).to(DEV)
    j = torch.from_numpy(np.ascontiguousarray(coo.j).view(np.int32)).to(DEV)
    k = torch.from_numpy(np.ascontiguousarray(coo.k).view(np.int32)).to(DEV)
    v = torch.from_numpy(np.ascontiguousarray(coo.val, dtype=np.float32)).to(DEV)
    return i, j, k, v


def build(ctx, coo, relabel=None, chunk_len=0):
    i, j, k, v = coo_to_dev(coo)
    t = dfacto.build_flattenings(ctx, coo.dims, i, j, k, v, relabel=relabel, chunk_len=chunk_len)
    torch.cuda.synchronize()
    return t


def factors_to_dev(factors, dtype="f32"):
    """FP64 host factors -> device tensors in the storage dtype, plus the
    same numbers widened to FP64 for the oracle."""
    out, widened = [], []
    for F in factors:
        f32 = np.ascontiguousarray(F, dtype=np.float32)
        if dtype == "f32":
            out.append(torch.from_numpy(f32.copy()).to(DEV))
            widened.append(f32.astype(np.float64))
        else:
            bits = gen.f32_to_bf16(f32)
            out.append(torch.from_numpy(bits.view(np.int16).copy()).to(DEV).view(torch.bfloat16))
            widened.append(gen.bf16_to_f32(bits).astype(np.float64))
    return out, widened


def to_host64(t: torch.Tensor) -> np.ndarray:
    return t.detach().float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 \
        else t.detach().cpu().numpy().astype(np.float64)


def rel_fro(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
