"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no part of the spline method: it only draws velocity fields
and particle positions.  Both the GPU path and the FP64 oracle receive the
same arrays from here.

Recipe (stand-in for the paper's DNS velocity fields, which are not available):
  * velocity: random Fourier modes on the integer wavevectors k with
    1 <= |k| <= kmax (|k| Euclidean); each mode gets a random complex vector
    projected perpendicular to k (divergence-free mode by mode) and scaled by
    |k|^(-11/6), so that shell energy goes as k^(-5/3); the real field is the
    real part of the inverse transform (equivalently the Hermitian-symmetrised
    spectrum); each component is then normalised to unit rms;
  * particles: uniform in the box [0, L)^3, or the clustered mix: the first
    half uniform, the second half in 64 Gaussian blobs (equal counts, centres
    uniform in the box, per-axis offsets N(0, sigma^2)), left unwrapped.
Seeds: field 0, uniform particles 1, blob centres and offsets 2, finite-
difference choices 4.
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def _wavenumbers(n):
    return np.fft.fftfreq(n, d=1.0 / n)  # integers in [-n/2, n/2)


def spectral_modes_np(n, kmax, seed=0):
    """Hermitian-symmetric spectrum uhat [3][n][n][n] (complex128, numpy FFT
    layout, axes (z, y, x)) such that field = ifftn(uhat) is real before
    normalisation.  Returns (uhat, scale) where field = scale[c] * ifftn(uhat[c])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k1 = _wavenumbers(n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    mask = (kk >= 1.0) & (kk <= kmax)
    a = rng.standard_normal((3, n, n, n)) + 1j * rng.standard_normal((3, n, n, n))
    kvec = np.stack([kx, ky, kz])
    with np.errstate(invalid="ignore", divide="ignore"):
        kdot = (kvec * a).sum(0) / np.where(kk > 0, kk * kk, 1.0)
    a = a - kvec * kdot
    amp = np.where(mask, np.power(np.where(kk > 0, kk, 1.0), -11.0 / 6.0), 0.0)
    a = a * amp
    # Hermitian symmetrisation: uhat(k) = (a(k) + conj(a(-k))) / 2
    neg = np.roll(np.flip(a, axis=(1, 2, 3)), shift=1, axis=(1, 2, 3))
    uhat = 0.5 * (a + np.conj(neg))
    field = np.fft.ifftn(uhat, axes=(1, 2, 3)).real
    rms = np.sqrt((field ** 2).mean(axis=(1, 2, 3)))
    return uhat, 1.0 / rms


def spectral_field_np(n, kmax, seed=0):
    """FP64 numpy velocity field [3][n][n][n] (x fastest), unit rms per component."""
    uhat, scale = spectral_modes_np(n, kmax, seed)
    field = np.fft.ifftn(uhat, axes=(1, 2, 3)).real
    return np.ascontiguousarray(field * scale[:, None, None, None])


def spectral_field_torch(n, kmax, seed=0, device="cuda"):
    """FP32 torch velocity field [3][n][n][n] on `device`, same recipe as the
    numpy generator (different random stream), built one component at a time
    with a half-spectrum inverse real FFT."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    kf = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float32)
    kh = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float32)
    kz = kf.view(n, 1, 1)
    ky = kf.view(1, n, 1)
    kx = kh.view(1, 1, -1)
    kk2 = kz * kz + ky * ky + kx * kx
    kk = kk2.sqrt()
    shape = (n, n, n // 2 + 1)
    a = [torch.complex(torch.randn(shape, generator=gen, device=device),
                       torch.randn(shape, generator=gen, device=device)) for _ in range(3)]
    inv = torch.where(kk2 > 0, 1.0 / kk2, torch.zeros_like(kk2))
    kdot = (kx * a[0] + ky * a[1] + kz * a[2]) * inv
    amp = torch.where((kk >= 1.0) & (kk <= kmax), kk.clamp_min(1.0).pow(-11.0 / 6.0),
                      torch.zeros_like(kk))
    comps = [(a[0] - kx * kdot) * amp, (a[1] - ky * kdot) * amp, (a[2] - kz * kdot) * amp]
    del a, kdot
    out = torch.empty((3, n, n, n), dtype=torch.float32, device=device)
    for c in range(3):
        f = torch.fft.irfftn(comps[c], s=(n, n, n), dim=(0, 1, 2))
        comps[c] = None
        f = f / f.square().mean().sqrt()
        out[c].copy_(f)
        del f
    return out


def spectral_field_torch_chunked(n, kmax, seed=0, device="cuda", chunk=128):
    """As spectral_field_torch for grids too large to hold three complex
    spectra at once (2048^3 needs 0.1 TB of device memory for the field alone):
    the random vectors of each slab of chunk kz-planes come from a generator
    seeded with (seed, slab), so every component can redraw them; the inverse
    transform runs one axis at a time over slabs.  Same spectrum and
    projection, a different random stream."""
    import torch

    kf = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float32)
    kh = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float32)
    nh = n // 2 + 1
    out = torch.empty((3, n, n, n), dtype=torch.float32, device=device)
    for c in range(3):
        spec = torch.empty((n, n, nh), dtype=torch.complex64, device=device)
        for z0 in range(0, n, chunk):
            z1 = min(n, z0 + chunk)
            gen = torch.Generator(device=device)
            gen.manual_seed(seed * 1000003 + z0)
            shape = (z1 - z0, n, nh)
            a = [torch.complex(torch.randn(shape, generator=gen, device=device),
                               torch.randn(shape, generator=gen, device=device))
                 for _ in range(3)]
            kz = kf[z0:z1].view(-1, 1, 1)
            ky = kf.view(1, n, 1)
            kx = kh.view(1, 1, nh)
            kk2 = kz * kz + ky * ky + kx * kx
            kk = kk2.sqrt()
            inv = torch.where(kk2 > 0, 1.0 / kk2, torch.zeros_like(kk2))
            kdot = (kx * a[0] + ky * a[1] + kz * a[2]) * inv
            amp = torch.where((kk >= 1.0) & (kk <= kmax), kk.clamp_min(1.0).pow(-11.0 / 6.0),
                              torch.zeros_like(kk))
            kc = (kx, ky, kz)[c]
            spec[z0:z1] = (a[c] - kc * kdot) * amp
            del a, kdot, kk2, kk, inv, amp
        for y0 in range(0, n, chunk):  # along z
            spec[:, y0:y0 + chunk] = torch.fft.ifft(spec[:, y0:y0 + chunk], dim=0)
        for z0 in range(0, n, chunk):  # along y, then the real transform along x
            blk = torch.fft.ifft(spec[z0:z0 + chunk], dim=1)
            out[c, z0:z0 + chunk] = torch.fft.irfft(blk, n=n, dim=2)
            del blk
        del spec
        ss = torch.zeros((), dtype=torch.float64, device=device)
        for z0 in range(0, n, chunk):
            ss += out[c, z0:z0 + chunk].double().square().sum()
        out[c] /= float((ss / float(n) ** 3).sqrt())
    return out


def uniform_particles_np(np_, L=TWO_PI, seed=1):
    """FP64 positions [3][np] uniform in [0, L)^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.random((3, np_)) * L)


def clustered_particles_np(np_, L=TWO_PI, sigma=0.1, nblobs=64, seed_uniform=1, seed_blob=2):
    """First half uniform in [0, L)^3, second half in `nblobs` Gaussian blobs
    of standard deviation sigma per axis around uniform centres (unwrapped)."""
    nu = np_ // 2
    nb = np_ - nu
    pos = np.empty((3, np_), dtype=np.float64)
    pos[:, :nu] = uniform_particles_np(nu, L, seed_uniform)
    rng = np.random.Generator(np.random.PCG64(seed_blob))
    centres = rng.random((3, nblobs)) * L
    owner = np.arange(nb) * nblobs // max(nb, 1)
    pos[:, nu:] = centres[:, owner] + sigma * rng.standard_normal((3, nb))
    return pos


def uniform_particles_torch(np_, L=TWO_PI, seed=1, device="cuda"):
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return torch.rand((3, np_), generator=gen, device=device, dtype=torch.float64) * L


def clustered_particles_torch(np_, L=TWO_PI, sigma=0.1, nblobs=64, seed_uniform=1,
                              seed_blob=2, device="cuda"):
    import torch

    nu = np_ // 2
    nb = np_ - nu
    pos = torch.empty((3, np_), dtype=torch.float64, device=device)
    pos[:, :nu] = uniform_particles_torch(nu, L, seed_uniform, device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed_blob)
    centres = torch.rand((3, nblobs), generator=gen, device=device, dtype=torch.float64) * L
    owner = torch.arange(nb, device=device) * nblobs // max(nb, 1)
    pos[:, nu:] = centres[:, owner] + sigma * torch.randn(
        (3, nb), generator=gen, device=device, dtype=torch.float64)
    return pos


def cfl_dt(field_max_abs, n, L=TWO_PI, courant=0.6):
    """Time step for which no particle moves more than `courant` grid
    spacings per step (the paper runs at Courant number 0.6)."""
    return courant * (L / n) / float(field_max_abs)
