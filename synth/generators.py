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


class SineWaveStream:
    """Noisy sine-wave stream with a rank bump (paper section 5.1, Fig. 3, Table 1).

    Two blocks of ``n_half`` slices sampled from
    f(x) = sum_j c_j sin(pi (j_1 x_1 + ... + j_d x_d)) on [-1, 1]^d (grid end
    points included, c_j i.i.d. N(0, 1)); the streaming coordinate x_d runs over
    its own uniform grid in each block. The first block keeps the terms with
    |j_d| <= f_a, the second all terms up to |j_d| <= f_b, with the same
    coefficients for the shared j, so the streaming-mode rank is 2 f_a + 1 over
    the first block and 2 f_b + 1 over the whole stream, and the spatial ranks
    are 2 f_k + 1 throughout. Gaussian noise, one seeded generator per slice, is
    scaled so that its norm over the whole stream is ``eta`` times that of the
    noise-free stream.

    The sum is evaluated in separable form: for each j_d the complex spatial
    field B_{j_d} = sum_{j_1..j_{d-1}} c_j prod_k exp(i pi j_k x_k), and a slice
    at coordinate s is Im(sum_{j_d} B_{j_d} exp(i pi j_d s)), which equals the
    sum of sines term by term.
    """

    def __init__(self, dims=(100, 100), n_half=2500, freqs=(5, 5), f_a=5, f_b=7,
                 eta=1e-3, seed=1005):
        self.dims = tuple(int(n) for n in dims)
        self.freqs = tuple(int(f) for f in freqs)
        self.n_half = int(n_half)
        self.n_slices = 2 * self.n_half
        self.f_a, self.f_b = int(f_a), int(f_b)
        self.eta = float(eta)
        self.seed = int(seed)
        rng = np.random.default_rng(seed)
        coef = rng.standard_normal(tuple(2 * f + 1 for f in self.freqs) + (2 * self.f_b + 1,))
        field = coef.astype(np.complex128)
        for ax, (n, f) in enumerate(zip(self.dims, self.freqs)):
            x = np.linspace(-1.0, 1.0, n)
            e = np.exp(1j * np.pi * np.outer(x, np.arange(-f, f + 1)))  # n x (2f+1)
            field = np.moveaxis(np.tensordot(e, field, axes=([1], [ax])), 0, ax)
        # columns: j_d = -f_b .. f_b; rows: the slice in column-major order
        self._basis = field.reshape(-1, 2 * self.f_b + 1, order="F")
        self._jd = np.arange(-self.f_b, self.f_b + 1)
        self._grid = np.linspace(-1.0, 1.0, self.n_half)
        sig2 = 0.0
        noise2 = 0.0
        for t in range(self.n_slices):
            sig2 += float(np.sum(self._clean(t) ** 2))
            noise2 += float(np.sum(self._noise_raw(t) ** 2))
        self.clean_norm = math.sqrt(sig2)
        self._noise_scale = self.eta * self.clean_norm / math.sqrt(noise2)

    def _clean(self, t):
        blk, i = divmod(int(t), self.n_half)
        keep = np.abs(self._jd) <= (self.f_a if blk == 0 else self.f_b)
        w = np.exp(1j * np.pi * self._jd[keep] * self._grid[i])
        return (self._basis[:, keep] @ w).imag

    def _noise_raw(self, t):
        return np.random.default_rng([self.seed, int(t)]).standard_normal(int(np.prod(self.dims)))

    def slice_flat(self, t):
        return self._clean(t) + self._noise_scale * self._noise_raw(t)

    def slice(self, t):
        return self.slice_flat(t).reshape(self.dims, order="F")

    def slice_torch(self, t, device, dtype):
        import torch
        return torch.from_numpy(self.slice_flat(t)).to(device=device, dtype=dtype)

    def expected_ranks(self):
        """Exact ranks of the noise-free stream: spatial, then the streaming mode
        over the first block and over the whole stream."""
        return tuple(2 * f + 1 for f in self.freqs), 2 * self.f_a + 1, 2 * self.f_b + 1


# The sine-wave experiment of paper section 5.1 (100 x 100 x 5000, rank bump at
# slice 2500, eta = 1e-3, tau = 1e-2, initial ST-HOSVD on 200 slices).
SINE_WAVE = dict(kind="sine", dims=(100, 100), n_half=2500, freqs=(5, 5), f_a=5, f_b=7,
                 eta=1e-3, eps=1e-2, n_init=200, seed=1005)

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
    if kind == "sine":
        return SineWaveStream(dims=c["dims"], n_half=c["n_half"], freqs=c["freqs"],
                              f_a=c["f_a"], f_b=c["f_b"], eta=c["eta"], seed=c["seed"])
    if kind == "fourier":
        return FourierStream(dims=c["dims"], n_modes=c.get("n_modes", 4096),
                             kmax=c.get("kmax", 64.0), drift=c.get("drift", 0.02),
                             n_slices=c["n_slices"], seed=c["seed"])
    raise ValueError(f"unknown stream kind {kind!r}")
