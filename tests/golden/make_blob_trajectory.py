"""Write the FP64 oracle's per-slice decisions on the 128^3 x 16 blob stream.

Runs only the oracle (no GPU code): ST-HOSVD of the first 20 slices, then the
streaming update of slices 20..399, on the float32 values of the slices (the
values the GPU library consumes), tau = 1e-4. Records after every slice the
ranks, eps, ||E_k||/eps per slice mode, q/eps, and the branch taken, so the GPU
run at full size can be compared decision by decision.

At checkpoints (every 50 updates and after the last slice) it also records the
oracle's reconstruction of probe slices {0, T//2, T} (T = the last slice seen)
at a fixed seeded sample of element positions, together with the data values
there, so a GPU run can be compared with the oracle element by element on
reconstructed slices (sampled outputs; the full slices would be 268 MB each).

With the argument ``factored`` the oracle keeps the core as C = V x_d S (its
core_update="factored"); the decisions are the same, the reconstructions of
the ignored residuals differ, and the output goes to a second file.

Usage: python tests/golden/make_blob_trajectory.py [n_slices] [literal|factored]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import StreamingTucker, vec  # noqa: E402
from synth import make_stream  # noqa: E402

N_SAMPLES = 1024
SAMPLE_SEED = 2024


def sample_positions(ny, n=N_SAMPLES, seed=SAMPLE_SEED):
    """Sorted distinct flat (column-major) element indices of a slice."""
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, ny, size=n)).astype(np.int64)


def main():
    n_slices = int(sys.argv[1]) if len(sys.argv) > 1 else 400
    core_update = sys.argv[2] if len(sys.argv) > 2 else "literal"
    s = make_stream(1)
    n_init, tau = 20, 1e-4
    ny = int(np.prod(s.dims))
    pos = sample_positions(ny)

    def flat32(t):
        return s.slice_flat(t).astype(np.float32).astype(np.float64)

    def sl(t):
        return flat32(t).reshape(s.dims, order="F")

    orc = StreamingTucker(np.stack([sl(t) for t in range(n_init)], axis=-1), tau,
                          core_update=core_update)
    vm = orc.vmat()
    init_v_orth = float(np.max(np.abs(vm.T @ vm - np.eye(vm.shape[1]))))
    out = dict(
        source="FP64 oracle (oracle/tucker.py), blob stream config 1, float32 slice values",
        core_update=core_update,
        stream=dict(space=list(s.space), n_vars=s.n_vars, n_blobs=s.n_blobs, seed=1001,
                    n_init=n_init, tau=tau, n_slices=n_slices),
        init_ranks=list(orc.ranks), init_bound=orc.recon_error_bound(), slices=[],
        probe_positions=pos.tolist(), probe_sample_seed=SAMPLE_SEED, checkpoints=[])
    checkpoints = set(range(n_init + 49, n_slices, 50)) | {n_slices - 1}
    t0 = time.time()
    for t in range(n_init, n_slices):
        rec = orc.update(sl(t))
        out["slices"].append(dict(
            t=t, ranks=list(orc.ranks), eps=rec["eps"],
            e_over_eps=[e / rec["eps"] for e in rec["e_norm"]], q_over_eps=rec["q"] / rec["eps"],
            grew=[int(g) for g in rec["r_new"]], ignored=bool(rec["ignored"]),
            bound=orc.recon_error_bound()))
        if t in checkpoints:
            probes = []
            for tp in sorted({0, t // 2, t}):
                rec_t = vec(orc.reconstruct_slice(tp))
                probes.append(dict(t=tp, recon=rec_t[pos].tolist(),
                                   data=flat32(tp)[pos].tolist(),
                                   slice_norm=float(np.linalg.norm(flat32(tp)))))
            out["checkpoints"].append(dict(after=t, probes=probes))
        print(t, orc.ranks, f"{time.time() - t0:.0f}s", flush=True)
    name = ("blobs128_oracle_trajectory.json" if core_update == "literal"
            else f"blobs128_oracle_trajectory_{core_update}.json")
    # how far the auxiliary V of the core factorization is from orthonormal
    # (the Gram-based SVD of Alg. 1 leaves about u (s_1 / s_r)^2)
    vm = orc.vmat()
    out["final_v_orth"] = float(np.max(np.abs(vm.T @ vm - np.eye(vm.shape[1]))))
    out["init_v_orth"] = init_v_orth
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
