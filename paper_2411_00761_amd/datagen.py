"""Seeded synthetic particle workloads (host, numpy PCG64).

These stand in for the paper's datasets (Tab. 1: MD trajectories such as Copper,
Helium, LJ and YIIP; the HACC cosmology snapshot), which are not available here.
This module holds no part of the compression method; it only draws inputs, and
both the GPU library's tests/benchmark and the CPU oracle consume the same arrays.
Every generator returns float32 structure-of-arrays data shaped (F, n), except
the fixed-point one, which returns int32 of the same shape.
"""
from __future__ import annotations

import numpy as np


def uniform_frame(n: int, lo: float = 0.0, hi: float = 100.0, seed: int = 1, F: int = 3):
    """n particles i.i.d. uniform in [lo, hi)^F."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, size=(F, n))
    return np.ascontiguousarray(np.minimum(x, np.nextafter(hi, lo)).astype(np.float32))


def lattice_dims(n: int):
    """A near-cubic lattice shape (nx >= ny >= nz) with nx*ny*nz >= n."""
    c = int(round(n ** (1.0 / 3.0)))
    for nz in range(max(1, c), 0, -1):
        ny = nz
        nx = -(-n // (ny * nz))
        if nx * ny * nz >= n:
            return nx, ny, nz
    return n, 1, 1


class MDTrajectory:
    """MD-like frames: particles on a cubic lattice with Gaussian jitter at t=0,
    then an independent Gaussian displacement per coordinate per step.  The
    particle order is lattice order (x fastest) and is the same in every frame."""

    def __init__(self, n: int, dims=None, spacing: float = 1.0, jitter: float = 0.1,
                 step: float = 0.01, seed: int = 2):
        self.n = n
        nx, ny, nz = dims if dims is not None else lattice_dims(n)
        self.rng = np.random.default_rng(seed)
        i = np.arange(n, dtype=np.int64)
        base = np.stack([(i % nx), (i // nx) % ny, i // (nx * ny)]).astype(np.float64) * spacing
        self.pos = base + self.rng.normal(0.0, jitter, size=(3, n))
        self.step = step
        self.t = 0

    def next_frame(self) -> np.ndarray:
        if self.t > 0:
            self.pos += self.rng.normal(0.0, self.step, size=self.pos.shape)
        self.t += 1
        return np.ascontiguousarray(self.pos.astype(np.float32))


def fixed_point(x: np.ndarray, units_per_length: float = 1000.0) -> np.ndarray:
    """Integer particle data: positions stored as int32 counts of a fixed length
    unit (e.g. 1e-3 of the lattice spacing), rounded to nearest."""
    return np.ascontiguousarray(np.rint(np.asarray(x, np.float64) * units_per_length)
                                .astype(np.int32))


def md_trajectory(n_frames: int, n: int = 1 << 22, dims=(256, 128, 128), seed: int = 2, **kw):
    traj = MDTrajectory(n, dims=dims, seed=seed, **kw)
    for _ in range(n_frames):
        yield traj.next_frame()


def clustered_positions(rng, n: int, box: float, n_halos: int, bg_frac: float,
                        sig_lo: float = 0.1, sig_hi: float = 2.0):
    """Gaussian halos (centres uniform in the box, sigma log-uniform) plus a uniform
    background, wrapped into [0, box), in shuffled order."""
    n_bg = int(round(bg_frac * n))
    n_h = n - n_bg
    centres = rng.uniform(0.0, box, size=(n_halos, 3))
    sig = np.exp(rng.uniform(np.log(sig_lo), np.log(sig_hi), size=n_halos))
    h = rng.integers(0, n_halos, size=n_h)
    pos = np.empty((3, n), np.float64)
    for d in range(3):
        pos[d, :n_h] = centres[h, d] + rng.normal(0.0, 1.0, size=n_h) * sig[h]
        pos[d, n_h:] = rng.uniform(0.0, box, size=n_bg)
    pos = np.mod(pos, box)
    perm = rng.permutation(n)
    out = np.empty((3, n), np.float32)
    for d in range(3):
        out[d] = np.minimum(pos[d, perm], np.nextafter(box, 0.0))
    return out


def cosmology_snapshot(n: int = 1 << 27, box: float = 256.0, n_halos: int = 2000,
                       bg_frac: float = 0.3, vel_sigma: float = 300.0, seed: int = 3):
    """Positions from halos + background, velocities N(0, vel_sigma^2): F = 6."""
    rng = np.random.default_rng(seed)
    out = np.empty((6, n), np.float32)
    out[:3] = clustered_positions(rng, n, box, n_halos, bg_frac)
    for d in range(3):
        out[3 + d] = rng.normal(0.0, vel_sigma, size=n).astype(np.float32)
    return out


def batched_sizes(n_frames: int = 256, lo_log2: int = 14, hi_log2: int = 22, seed: int = 4):
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(lo_log2 * np.log(2), hi_log2 * np.log(2),
                                       size=n_frames))).astype(np.int64)


def batched_frames(n_frames: int = 256, lo_log2: int = 14, hi_log2: int = 22, seed: int = 4):
    """Independent frames of log-uniform size; even frames uniform in [0,100)^3,
    odd frames clustered (200 halos, 30% background) in [0,100)^3."""
    sizes = batched_sizes(n_frames, lo_log2, hi_log2, seed)
    rng = np.random.default_rng(seed + 1000)
    frames = []
    for j, n in enumerate(sizes):
        if j % 2 == 0:
            frames.append(np.minimum(rng.uniform(0.0, 100.0, size=(3, n)),
                                     np.nextafter(100.0, 0.0)).astype(np.float32))
        else:
            frames.append(clustered_positions(rng, int(n), 100.0, 200, 0.3))
    return frames


def serve_stream_sizes(n_streams: int = 32, lo_log2: int = 16, hi_log2: int = 24, seed: int = 5):
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(lo_log2 * np.log(2), hi_log2 * np.log(2),
                                       size=n_streams))).astype(np.int64)


def poisson_arrivals(rate_hz: float, n: int, seed: int = 5):
    rng = np.random.default_rng(seed + 7)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def cosmology_snapshot_device(torch, n: int = 1 << 27, device="cuda", box: float = 256.0,
                              n_halos: int = 2000, bg_frac: float = 0.3, vel_sigma: float = 300.0,
                              seed: int = 3):
    """The cosmology-like snapshot's recipe drawn on the device with torch's
    generator (same distributions as cosmology_snapshot, other random numbers):
    70% of the particles in Gaussian halos (centres uniform in the box, sigma
    log-uniform in [0.1, 2.0], halo chosen uniformly), 30% uniform, wrapped into
    [0, box), shuffled; velocities N(0, vel_sigma^2).  Returns a (6, n) float32
    tensor."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n_bg = int(round(bg_frac * n))
    n_h = n - n_bg
    centres = torch.rand((n_halos, 3), generator=g, device=device, dtype=torch.float64) * box
    sig = torch.exp(torch.rand(n_halos, generator=g, device=device, dtype=torch.float64)
                    * (np.log(2.0) - np.log(0.1)) + np.log(0.1))
    h = torch.randint(0, n_halos, (n_h,), generator=g, device=device)
    out = torch.empty((6, n), dtype=torch.float32, device=device)
    perm = torch.randperm(n, generator=g, device=device)
    top = float(np.nextafter(np.float32(box), np.float32(0.0)))
    for d in range(3):
        pos = torch.empty(n, dtype=torch.float64, device=device)
        pos[:n_h] = centres[h, d] + torch.randn(n_h, generator=g, device=device,
                                                dtype=torch.float64) * sig[h]
        pos[n_h:] = torch.rand(n_bg, generator=g, device=device, dtype=torch.float64) * box
        pos = torch.remainder(pos, box)
        out[d] = torch.clamp(pos[perm].to(torch.float32), max=top)
        del pos
    for d in range(3):
        out[3 + d] = torch.randn(n, generator=g, device=device, dtype=torch.float32) * vel_sigma
    return out
