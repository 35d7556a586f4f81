"""Helpers shared by the GPU parity tests: host <-> device copies that keep
column-major storage, and error measures."""
import numpy as np
import torch


def to_dev(a: np.ndarray, dtype=None, device="cuda") -> torch.Tensor:
    a = np.asarray(a)
    if a.ndim == 1:
        t = torch.from_numpy(np.ascontiguousarray(a))
        return t.to(device=device, dtype=dtype) if dtype is not None else t.to(device)
    f = np.asfortranarray(a)
    host = torch.from_numpy(f.T.copy(order="C")).t()  # column-major view of a copy
    tdt = dtype if dtype is not None else host.dtype
    out = torch.empty((a.shape[1], a.shape[0]), dtype=tdt, device=device).t()
    out.copy_(host)
    return out


def bf16_dev(values_f32: np.ndarray, device="cuda") -> torch.Tensor:
    """A column-major torch.bfloat16 device tensor holding BF16-representable
    float32 values exactly."""
    t = to_dev(np.asarray(values_f32, dtype=np.float32), device=device)
    out = torch.empty((t.shape[1], t.shape[0]), dtype=torch.bfloat16, device=device).t()
    out.copy_(t)  # exact: the values are representable
    return out


def f16_dev(values_f32: np.ndarray, device="cuda") -> torch.Tensor:
    """A column-major torch.float16 device tensor holding FP16-representable
    float32 values exactly."""
    t = to_dev(np.asarray(values_f32, dtype=np.float32), device=device)
    out = torch.empty((t.shape[1], t.shape[0]), dtype=torch.float16, device=device).t()
    out.copy_(t)  # exact: the values are representable
    return out


def g_dev(G: np.ndarray, gd: str, device="cuda") -> torch.Tensor:
    """G on the device in the stored format named by gd (f64, f32, bf16, f16)."""
    if gd == "bf16":
        return bf16_dev(G, device)
    if gd == "f16":
        return f16_dev(G, device)
    return to_dev(G, device=device)


def to_host(t: torch.Tensor) -> np.ndarray:
    if t.dim() == 1:
        return t.detach().cpu().numpy()
    return np.asfortranarray(t.detach().cpu().numpy())


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def bits_equal(a: np.ndarray, b: np.ndarray) -> bool:
    """Bitwise equality (distinguishes +0.0 from -0.0)."""
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    if a.dtype != b.dtype or a.shape != b.shape:
        return False
    u = np.uint64 if a.dtype == np.float64 else np.uint32
    return bool(np.array_equal(a.view(u), b.view(u)))
