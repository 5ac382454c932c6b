"""Shared helpers for the GPU parity tests (GPU path vs the FP64 oracle)."""

from __future__ import annotations

import numpy as np

from oracle import StreamingTucker as Oracle
from oracle import vec


def slices32(stream, count):
    """float32 slices (flat, column-major) and the same values as float64 arrays."""
    flat = [stream.slice_flat(t).astype(np.float32) for t in range(count)]
    shaped = [f.astype(np.float64).reshape(stream.dims, order="F") for f in flat]
    return flat, shaped


def margins(rec):
    """Smallest relative distance of the slice's threshold tests from eps."""
    eps = rec["eps"]
    if eps == 0:
        return np.inf
    vals = [abs(e / eps - 1.0) for e in rec["e_norm"]] + [abs(rec["q"] / eps - 1.0)]
    return min(vals)


def run_parity(stream, n_slices, n_init, tau, precision="fp32", err_tol=1e-5,
               probe_every=1, marginal=1e-3, guard_rel=0.0, core_update="literal",
               orth_tol=0.0, eps_m=1e-12):
    """Stream the same float32 slices through the GPU path and the oracle.

    Returns a dict with the per-slice rank sequences, the worst error of the GPU
    reconstruction against the oracle's (relative to ||Y_t||), the slice where
    the ranks first differed (None if never) and the oracle margin there.
    """
    import torch

    import paper_2308_16395_amd as pkg

    flat, shaped = slices32(stream, n_slices)
    x0 = np.concatenate(flat[:n_init])
    orc = Oracle(np.stack(shaped[:n_init], axis=-1), tau, core_update=core_update, eps_m=eps_m)
    gpu = pkg.StreamingTucker(stream.dims, tau, precision=precision, guard_rel=guard_rel,
                              core_update=core_update, orth_tol=orth_tol)
    gpu.init(torch.from_numpy(x0).cuda(), n_init)
    out = dict(gpu_ranks=[gpu.ranks], orc_ranks=[orc.ranks], worst_err=0.0, diverged_at=None,
               margin_at_divergence=None, stats=[])
    if gpu.ranks != orc.ranks:
        out["diverged_at"] = n_init - 1
        return out, gpu, orc
    for t in range(n_init, n_slices):
        y = torch.from_numpy(flat[t]).cuda()
        gpu.update(y)
        rec = orc.update(shaped[t])
        out["gpu_ranks"].append(gpu.ranks)
        out["orc_ranks"].append(orc.ranks)
        out["stats"].append(gpu.stats())
        if gpu.ranks != orc.ranks:
            out["diverged_at"] = t
            out["margin_at_divergence"] = margins(rec)
            break
        if (t - n_init) % probe_every == 0 or t == n_slices - 1:
            ynorm = np.linalg.norm(shaped[t])
            for probe in sorted({t, (t + n_init) // 2, 0}):
                g = gpu.reconstruct_slice(probe).cpu().numpy().astype(np.float64)
                o = vec(orc.reconstruct_slice(probe))
                yn = np.linalg.norm(shaped[probe]) if probe != t else ynorm
                out["worst_err"] = max(out["worst_err"], np.linalg.norm(g - o) / yn)
    return out, gpu, orc
