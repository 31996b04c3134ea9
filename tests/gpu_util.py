"""Helpers shared by the GPU tests (device grids, padded layouts, seeds)."""
import numpy as np
import torch

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def dev_grid(a: np.ndarray, ld: int | None = None, dtype=torch.float64, pad_value=float("nan")):
    """Copy a (ny, nx) array to the GPU, optionally inside a wider (ny, ld)
    buffer whose extra columns hold pad_value."""
    ny, nx = a.shape
    if ld is None or ld == nx:
        return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)
    buf = torch.full((ny, ld), pad_value, dtype=dtype, device=DEV)
    buf[:, :nx] = torch.from_numpy(a).to(DEV, dtype)
    return buf[:, :nx]


def empty_like_grid(t: torch.Tensor, dtype=None, pad_value=float("nan")):
    ny, nx = t.shape
    ld = t.stride(0)
    buf = torch.full((ny, ld), pad_value, dtype=dtype or t.dtype, device=t.device)
    return buf[:, :nx]


def padding_intact(t: torch.Tensor, pad_value=float("nan")) -> bool:
    ny, nx = t.shape
    ld = t.stride(0)
    if ld == nx:
        return True
    full = torch.as_strided(t, (ny, ld), (ld, 1))
    pad = full[:, nx:]
    if pad_value != pad_value:
        return bool(torch.isnan(pad).all())
    return bool((pad == pad_value).all())


def smooth_data(nx, ny, seed):
    from paper_1904_04048_amd.workloads import random_modes, sine_series
    rng = np.random.Generator(np.random.PCG64(seed))
    kmax = max(1, min(8, nx - 2, ny - 2))
    ms = random_modes(rng, count=min(8, kmax * kmax), kmax=kmax)
    return sine_series(nx, ny, ms), ms


def rough_data(nx, ny, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx))
