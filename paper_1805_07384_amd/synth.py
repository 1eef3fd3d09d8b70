"""Seeded synthetic inputs shaped like the paper's workloads.

The paper evaluates on NYX (3D 2048^3 cosmology), CESM-ATM (2D 1800x3600
climate) and Hurricane (3D 100x500x500) fields (Table 1).  Those data sets are
not available here; seeded Gaussian random fields (GRFs) with power-law
spectra stand in for them.  This module holds no part of the compression
method: it only produces inputs, identically for the GPU library and for the
CPU oracle (both receive the same array).

Recipe (every generator is deterministic in its seed):
  white N(0,1) noise -> real FFT -> amplitude * k^(alpha/2) with k the
  wavevector magnitude in cycles/sample and the k = 0 mode zeroed -> inverse
  FFT -> normalised to zero mean, unit variance.
"""
from __future__ import annotations

import math

import numpy as np


def _kgrid_np(shape):
    axes = []
    for i, n in enumerate(shape):
        if i == len(shape) - 1:
            axes.append(np.fft.rfftfreq(n))
        else:
            axes.append(np.fft.fftfreq(n))
    grids = np.meshgrid(*axes, indexing="ij", sparse=True)
    k2 = sum(g * g for g in grids)
    return np.sqrt(k2)


def grf_numpy(shape, alpha: float, seed: int) -> np.ndarray:
    """Unit-variance GRF (float64) with power spectrum ~ k^alpha, on the CPU."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    if noise.size == 1:
        return np.zeros(shape)
    f = np.fft.rfftn(noise)
    k = _kgrid_np(shape)
    with np.errstate(divide="ignore"):
        amp = np.where(k > 0, k ** (alpha / 2.0), 0.0)
    g = np.fft.irfftn(f * amp, s=shape, axes=tuple(range(len(shape))))
    g -= g.mean()
    sd = g.std()
    return g / sd if sd > 0 else g


def grf_torch(shape, alpha: float, seed: int, device="cuda", dtype=None):
    """Same recipe on a torch device (used for the large benchmark fields)."""
    import torch

    dtype = dtype or torch.float64
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    noise = torch.randn(tuple(shape), generator=gen, device=device, dtype=dtype)
    f = torch.fft.rfftn(noise)
    del noise
    k2 = None
    for i, n in enumerate(shape):
        if i == len(shape) - 1:
            ax = torch.fft.rfftfreq(n, device=device, dtype=dtype)
        else:
            ax = torch.fft.fftfreq(n, device=device, dtype=dtype)
        view = [1] * len(shape)
        view[i] = ax.numel()
        a2 = (ax * ax).reshape(view)
        k2 = a2 if k2 is None else k2 + a2
    k = torch.sqrt(k2)
    amp = torch.where(k > 0, k.clamp_min(1e-300) ** (alpha / 2.0), torch.zeros_like(k))
    f.mul_(amp)
    del amp, k, k2
    g = torch.fft.irfftn(f, s=tuple(shape))
    del f
    g -= g.mean()
    g /= g.std()
    return g


def affine_to_range(g, lo: float, hi: float):
    """Map [min g, max g] affinely onto [lo, hi] (float64 arithmetic)."""
    gmin = float(g.min())
    gmax = float(g.max())
    scale = (hi - lo) / (gmax - gmin) if gmax > gmin else 0.0
    return (g - gmin) * scale + lo


# -- the benchmark configurations -------------------------------------------

def field_2d_grf(ny=512, nx=512, seed=1, backend="numpy", device="cuda"):
    """2D float32 GRF, spectrum ~k^-3, affinely mapped onto [-50, 50]."""
    if backend == "numpy":
        g = grf_numpy((ny, nx), -3.0, seed)
        return affine_to_range(g, -50.0, 50.0).astype(np.float32)
    import torch
    g = grf_torch((ny, nx), -3.0, seed, device=device)
    return affine_to_range(g, -50.0, 50.0).to(torch.float32)


def field_3d_lognormal(n=512, seed=2, backend="numpy", device="cuda", shape=None):
    """3D float32 field exp(g): g a unit-variance GRF with spectrum ~k^(-11/3),
    so the field is a lognormal(0, 1) multiplicative density contrast."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    if backend == "numpy":
        return np.exp(grf_numpy(shape, -11.0 / 3.0, seed)).astype(np.float32)
    import torch
    g = grf_torch(shape, -11.0 / 3.0, seed, device=device, dtype=torch.float32)
    return torch.exp(g)


def field_3d_spiky_f64(n=1024, seed=5, backend="numpy", device="cuda", shape=None,
                       spike_frac=0.01, spike_mag=1e3):
    """3D float64 GRF (spectrum ~k^-3, sigma 1) plus Bernoulli(spike_frac)
    spikes of magnitude spike_mag * sigma with random sign."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    if backend == "numpy":
        g = grf_numpy(shape, -3.0, seed)
        rng = np.random.default_rng(seed + 7919)
        m = rng.random(shape) < spike_frac
        sgn = np.where(rng.random(shape) < 0.5, -1.0, 1.0)
        return np.where(m, g + sgn * spike_mag, g)
    import torch
    g = grf_torch(shape, -3.0, seed, device=device, dtype=torch.float64)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) + 7919)
    u = torch.rand(shape, generator=gen, device=device, dtype=torch.float64)
    m = u < spike_frac
    del u
    s = torch.rand(shape, generator=gen, device=device, dtype=torch.float64)
    g = torch.where(m, g + torch.where(s < 0.5, -spike_mag, spike_mag), g)
    return g


def batch_fields_spec(n_fields=120, seed=3):
    """Per-field parameters of the batched workload: spectral slope
    alpha ~ U[-4, -2], value range 10^U(-3, 4), target PSNR ~ U[40, 120]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_fields):
        alpha = float(rng.uniform(-4.0, -2.0))
        rng_exp = float(rng.uniform(-3.0, 4.0))
        psnr = float(rng.uniform(40.0, 120.0))
        out.append({"seed": seed * 100003 + i, "alpha": alpha, "range": 10.0 ** rng_exp,
                    "psnr": psnr})
    return out


def batch_field(spec, shape=(1800, 3600), backend="numpy", device="cuda"):
    r = spec["range"]
    if backend == "numpy":
        g = grf_numpy(shape, spec["alpha"], spec["seed"])
        return affine_to_range(g, -r / 2, r / 2).astype(np.float32)
    import torch
    g = grf_torch(shape, spec["alpha"], spec["seed"], device=device)
    return affine_to_range(g, -r / 2, r / 2).to(torch.float32)


def serve_trace(n_req=2000, rate=200.0, seed=4, median_bytes=16 << 20, sigma_ln=1.0,
                min_bytes=1 << 20, max_bytes=2 << 30, compress_frac=0.7):
    """Seeded request trace: Poisson arrivals, 70/30 compress/decompress,
    lognormal request size clipped to [1 MiB, 2 GiB], 1D/2D/3D shapes,
    targets ~ U[40, 120] dB."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n_req):
        t += float(rng.exponential(1.0 / rate))
        kind = "compress" if rng.random() < compress_frac else "decompress"
        size = float(np.exp(np.log(median_bytes) + sigma_ln * rng.standard_normal()))
        size = int(min(max(size, min_bytes), max_bytes))
        n = max(1, size // 4)
        nd = int(rng.integers(1, 4))
        if nd == 1:
            shape = (n,)
        elif nd == 2:
            h = max(1, int(math.sqrt(n / 2)))
            shape = (h, max(1, n // h))
        else:
            c = max(1, int(round(n ** (1 / 3))))
            shape = (c, c, max(1, n // (c * c)))
        reqs.append({"id": i, "t": t, "kind": kind, "shape": shape,
                     "psnr": float(rng.uniform(40.0, 120.0)), "seed": seed * 1000003 + i,
                     "pick": float(rng.random())})
    return reqs


def periodic_bases(alpha: float = -3.0, seed: int = 9, device="cuda",
                   sizes=((1 << 22,), (2048, 2048), (128, 128, 128))):
    """One unit-variance float32 GRF per dimensionality (power-of-two
    periodic boxes), from which request fields of any shape are cut."""
    return {len(sh): grf_torch(sh, alpha, seed + len(sh), device=device).float()
            for sh in sizes}


def periodic_crop(bases, shape, seed: int):
    """A field of ``shape`` cut from the periodic extension of the base GRF of
    its dimensionality at a seeded offset.  A GRF made by FFT is periodic, so
    the tiling has no seams; structure repeats every base length."""
    import torch

    base = bases[len(shape)]
    rng = np.random.default_rng(seed)
    off = [int(rng.integers(0, b)) for b in base.shape]
    reps = [-(-(o + n) // b) for o, n, b in zip(off, shape, base.shape)]
    t = base.repeat(*reps)
    sl = tuple(slice(o, o + n) for o, n in zip(off, shape))
    return t[sl].contiguous() if t.dtype == torch.float32 else t[sl].float().contiguous()

