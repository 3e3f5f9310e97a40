"""Shared helpers for the GPU parity tests (inputs from smc_inputs, expectations from oracle)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda")


def lib():
    import paper_2601_21983_amd as P  # raises ImportError if libsmc.so is missing
    return P


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda").contiguous()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def bf16_round(a):
    """Inputs rounded to the nearest BF16 value (ties to even), returned as float64.

    Split-BF16 GEMMs read the data as one BF16 value; the oracle evaluated on these
    rounded inputs is the exact quantity that mode approximates."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
