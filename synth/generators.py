"""Synthetic slice streams (input data only; no Tucker arithmetic here).

Each stream has ``dims`` (the slice shape n_1..n_{d-1}), ``n_slices`` and
``slice(t)`` returning a float64 Fortran-order array of shape ``dims``.
``slice_flat(t)`` returns the same values as a flat float64 vector in
column-major order, which is the memory layout the GPU library consumes.
"""

from __future__ import annotations

import math

import numpy as np


def _orthonormal(rng, m, r):
    q, _ = np.linalg.qr(rng.standard_normal((m, r)))
    return q


class LowRankStream:
    """Exactly low-rank 3-way tensor plus Gaussian noise, streamed on mode 3.

    X = G x_1 A x_2 B x_3 C with a Gaussian core G of shape ``ranks`` and random
    orthonormal A, B, C; noise is i.i.d. N(0, sigma^2) with
    sigma = noise_rel * ||X_clean||_F / sqrt(numel).
    The whole tensor is small, so it is materialised once.
    """

    def __init__(self, dims=(32, 32), n_slices=100, ranks=(4, 4, 6),
                 noise_rel=1e-4, seed=1000):
        rng = np.random.default_rng(seed)
        self.dims = tuple(int(n) for n in dims)
        self.n_slices = int(n_slices)
        self.ranks = tuple(ranks)
        core = rng.standard_normal(ranks)
        a = _orthonormal(rng, self.dims[0], ranks[0])
        b = _orthonormal(rng, self.dims[1], ranks[1])
        c = _orthonormal(rng, self.n_slices, ranks[2])
        clean = np.einsum("abc,ia,jb,tc->ijt", core, a, b, c, optimize=True)
        self.clean_norm = float(np.linalg.norm(clean))
        sigma = noise_rel * self.clean_norm / math.sqrt(clean.size)
        self.noise_sigma = sigma
        noise = sigma * rng.standard_normal(clean.shape) if noise_rel > 0 else 0.0
        self.full = np.asfortranarray(clean + noise)

    def slice(self, t):
        return np.asfortranarray(self.full[:, :, t])

    def slice_flat(self, t):
        return self.slice(t).ravel(order="F")


class BlobStream:
    """Advecting Gaussian blobs on a periodic 3-D grid, several variables.

    Slice t has shape (n_x, n_y, n_z, n_vars). Blob b has a centre c_b (uniform
    in the box), an isotropic width s_b (uniform in ``width`` cells), a velocity
    w_b (uniform in [-speed, speed] cells per slice on each axis); variable v
    carries blob b with amplitude a_{v,b} (uniform in ``amp``). With the periodic
    minimum-image offset dx,

        Y_t(x, v) = sum_b a_{v,b} prod_axis exp(-dx(x_ax, c_b,ax + w_b,ax t)^2 / (2 s_b^2)).

    Each blob is separable, so a slice is a sum of ``n_blobs`` outer products.
    """

    def __init__(self, space=(128, 128, 128), n_vars=16, n_blobs=32,
                 width=(4.0, 16.0), speed=0.5, amp=(0.1, 10.0), n_slices=400,
                 seed=1001):
        rng = np.random.default_rng(seed)
        self.space = tuple(int(n) for n in space)
        self.n_vars = int(n_vars)
        self.dims = self.space + ((self.n_vars,) if self.n_vars > 1 else ())
        self.n_slices = int(n_slices)
        self.n_blobs = int(n_blobs)
        ext = np.array(self.space, dtype=np.float64)
        self.center = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * ext
        self.width = rng.uniform(width[0], width[1], size=n_blobs)
        self.vel = rng.uniform(-speed, speed, size=(n_blobs, 3))
        self.amp = rng.uniform(amp[0], amp[1], size=(self.n_vars, n_blobs))

    def profiles(self, t):
        """Per-axis blob profiles g[ax] of shape (n_blobs, n_ax) at slice t."""
        out = []
        for ax, n in enumerate(self.space):
            x = np.arange(n, dtype=np.float64)
            c = self.center[:, ax] + self.vel[:, ax] * t
            dx = x[None, :] - c[:, None]
            dx = dx - n * np.round(dx / n)
            out.append(np.exp(-dx * dx / (2.0 * self.width[:, None] ** 2)))
        return out

    def slice_flat(self, t):
        g0, g1, g2 = self.profiles(t)
        # M[b, v, k, j] = g1[b, j] g2[b, k] amp[v, b]; rows of the mode-1
        # unfolding are then g0^T M with the column index j + n_y (k + n_z v).
        m = (self.amp.T[:, :, None, None] * g2[:, None, :, None]
             * g1[:, None, None, :])
        m = m.reshape(self.n_blobs, -1)
        return np.ascontiguousarray((m.T @ g0).ravel())

    def slice(self, t):
        return self.slice_flat(t).reshape(self.dims, order="F")

    def slice_torch(self, t, device, dtype):
        """Same values assembled on a torch device (input staging only)."""
        import torch

        g0, g1, g2 = (torch.from_numpy(g).to(device) for g in self.profiles(t))
        amp = torch.from_numpy(self.amp).to(device)
        m = (amp.T[:, :, None, None] * g2[:, None, :, None] * g1[:, None, None, :])
        m = m.reshape(self.n_blobs, -1)
        return (m.T @ g0).reshape(-1).to(dtype)


class FourierStream:
    """Random-Fourier field with a k^(-5/3) shell spectrum and phase drift.

    ``n_modes`` wave-vectors with |k| uniform in [1, kmax] and a uniform random
    direction, rounded to integers (zero vectors dropped); amplitude |k|^(-5/6),
    phase uniform in [0, 2 pi), per-slice drift omega = drift * |k|^(2/3).
    Y_t(x) = sum_j A_j cos(2 pi sum_ax k_ax x_ax / n_ax + phi_j + omega_j t),
    scaled by a fixed constant so that the field has RMS about 1.
    """

    def __init__(self, dims=(512, 512, 256), n_modes=4096, kmax=64.0,
                 drift=0.02, n_slices=1000, seed=1004):
        rng = np.random.default_rng(seed)
        self.dims = tuple(int(n) for n in dims)
        self.n_slices = int(n_slices)
        kmag = rng.uniform(1.0, kmax, size=n_modes)
        direc = rng.standard_normal((n_modes, 3))
        direc /= np.linalg.norm(direc, axis=1, keepdims=True)
        k = np.rint(direc * kmag[:, None]).astype(np.int64)
        keep = np.any(k != 0, axis=1)
        self.k = k[keep]
        kn = np.linalg.norm(self.k.astype(np.float64), axis=1)
        self.amp = kn ** (-5.0 / 6.0)
        self.phase = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)[keep]
        self.omega = drift * kn ** (2.0 / 3.0)
        self.scale = 1.0 / math.sqrt(0.5 * float(np.sum(self.amp ** 2)))

    def _spectrum_index(self):
        n = self.dims
        return tuple(np.mod(self.k[:, ax], n[ax]) for ax in range(3))

    def slice(self, t):
        n = self.dims
        spec = np.zeros(n, dtype=np.complex128)
        coef = self.amp * np.exp(1j * (self.phase + self.omega * t))
        np.add.at(spec, self._spectrum_index(), coef)
        field = np.fft.ifftn(spec).real * float(np.prod(n))
        return np.asfortranarray(self.scale * field)

    def slice_flat(self, t):
        return self.slice(t).ravel(order="F")

    def slice_torch(self, t, device, dtype):
        import torch

        n = self.dims
        spec = torch.zeros(n, dtype=torch.complex128, device=device)
        coef = self.amp * np.exp(1j * (self.phase + self.omega * t))
        idx = [torch.from_numpy(i).to(device) for i in self._spectrum_index()]
        spec.index_put_(tuple(idx), torch.from_numpy(coef).to(device), accumulate=True)
        field = torch.fft.ifftn(spec).real * float(np.prod(n)) * self.scale
        # field[i0, i1, i2] -> column-major flat order (i0 fastest)
        return field.permute(2, 1, 0).contiguous().reshape(-1).to(dtype)


class SineWaveTensor:
    """Sampled sum of sines on a uniform grid of [-1, 1]^d (paper section 5.1).

    f(x) = sum_{j_1=-f_1..f_1} ... sum_{j_d=-f_d..f_d} c_j sin(pi (j_1 x_1 + ... + j_d x_d)),
    with c_j i.i.d. N(0, 1) (the paper does not state their law). The grid
    includes both end points. By the angle-sum identities the mode-k
    unfolding has rank 2 f_k + 1.
    """

    def __init__(self, dims=(20, 20, 30), freqs=(1, 2, 3), seed=7):
        rng = np.random.default_rng(seed)
        self.dims = tuple(int(n) for n in dims)
        self.freqs = tuple(int(f) for f in freqs)
        grids = np.meshgrid(*[np.linspace(-1.0, 1.0, n) for n in self.dims],
                            indexing="ij")
        js = np.meshgrid(*[np.arange(-f, f + 1) for f in self.freqs], indexing="ij")
        js = np.stack([j.ravel() for j in js], axis=1)
        coef = rng.standard_normal(js.shape[0])
        full = np.zeros(self.dims)
        for c, j in zip(coef, js):
            arg = sum(float(j[ax]) * grids[ax] for ax in range(len(self.dims)))
            full += c * np.sin(np.pi * arg)
        self.full = np.asfortranarray(full)

    def expected_ranks(self):
        return tuple(2 * f + 1 for f in self.freqs)


# The five workloads the benchmark and the parity tests use (0-indexed).
CONFIGS = {
    0: dict(kind="lowrank", dims=(32, 32), n_slices=100, ranks=(4, 4, 6),
            noise_rel=1e-4, eps=1e-3, n_init=10, seed=1000),
    1: dict(kind="blobs", space=(128, 128, 128), n_vars=16, n_blobs=32,
            n_slices=400, eps=1e-4, n_init=20, seed=1001, precision="fp32"),
    2: dict(kind="blobs", space=(128, 128, 128), n_vars=16, n_blobs=32,
            n_slices=400, eps=1e-4, n_init=20, seed=1001, precision="bf16x3"),
    3: dict(kind="blobs", space=(96, 96, 96), n_vars=8, n_blobs=32,
            n_slices=16, ranks=(24, 24, 24, 6, 8), seed=1003),
    4: dict(kind="fourier", dims=(512, 512, 256), n_slices=1000, eps=1e-4,
            n_init=20, seed=1004),
}


def make_stream(cfg, **overrides):
    """Build the stream of a workload, optionally at other sizes."""
    c = dict(CONFIGS[cfg]) if isinstance(cfg, int) else dict(cfg)
    c.update(overrides)
    kind = c["kind"]
    if kind == "lowrank":
        return LowRankStream(dims=c["dims"], n_slices=c["n_slices"],
                             ranks=c["ranks"], noise_rel=c["noise_rel"],
                             seed=c["seed"])
    if kind == "blobs":
        return BlobStream(space=c["space"], n_vars=c["n_vars"],
                          n_blobs=c.get("n_blobs", 32),
                          width=c.get("width", (4.0, 16.0)),
                          speed=c.get("speed", 0.5), n_slices=c["n_slices"],
                          seed=c["seed"])
    if kind == "fourier":
        return FourierStream(dims=c["dims"], n_modes=c.get("n_modes", 4096),
                             kmax=c.get("kmax", 64.0), drift=c.get("drift", 0.02),
                             n_slices=c["n_slices"], seed=c["seed"])
    raise ValueError(f"unknown stream kind {kind!r}")
