"""Write the FP64 oracle's decisions on the first updates of the 512 x 512 x 256
random-Fourier stream (tau = 1e-4, initial ST-HOSVD on 20 slices).

Runs only the oracle (no GPU code) on the float32 values of the slices (the
values the GPU library consumes). Records after every update the ranks, eps,
||E_k||/eps per slice mode, q/eps and the branch taken, and at checkpoints the
oracle's reconstruction of probe slices {0, T//2, T} at a fixed seeded sample
of element positions (with the data there), as the blob-stream script does.
A full 1000-slice oracle run does not fit a test; the first updates carry the
initial growth of every mode.

With the second argument ``factored`` the oracle keeps the core as C = V x_d S
and the output goes to a second file (same decisions, different probes).

Usage: python tests/golden/make_fourier_trajectory.py [n_updates] [literal|factored]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

from make_blob_trajectory import sample_positions  # noqa: E402
from oracle import StreamingTucker, vec  # noqa: E402
from synth import CONFIGS, make_stream  # noqa: E402


def main():
    n_updates = int(sys.argv[1]) if len(sys.argv) > 1 else 40
    core_update = sys.argv[2] if len(sys.argv) > 2 else "literal"
    cfg = CONFIGS[4]
    s = make_stream(4)
    n_init, tau = cfg["n_init"], cfg["eps"]
    n_slices = n_init + n_updates
    ny = int(np.prod(s.dims))
    pos = sample_positions(ny)

    def flat32(t):
        return s.slice_flat(t).astype(np.float32).astype(np.float64)

    t0 = time.time()
    x0 = np.empty(s.dims + (n_init,), dtype=np.float64, order="F")
    for t in range(n_init):
        x0[..., t] = flat32(t).reshape(s.dims, order="F")
    orc = StreamingTucker(x0, tau, core_update=core_update)
    del x0
    vm = orc.vmat()
    init_v_orth = float(np.max(np.abs(vm.T @ vm - np.eye(vm.shape[1]))))
    print("init", orc.ranks, f"{time.time() - t0:.0f}s", init_v_orth, flush=True)
    out = dict(
        source="FP64 oracle (oracle/tucker.py), random-Fourier stream config 4, float32 "
               "slice values",
        core_update=core_update,
        stream=dict(dims=list(s.dims), n_init=n_init, tau=tau, n_slices=n_slices,
                    seed=cfg["seed"]),
        init_ranks=list(orc.ranks), init_bound=orc.recon_error_bound(), slices=[],
        probe_positions=pos.tolist(), checkpoints=[])
    checkpoints = {n_init + n_updates // 2 - 1, n_slices - 1}
    for t in range(n_init, n_slices):
        rec = orc.update(flat32(t).reshape(s.dims, order="F"))
        out["slices"].append(dict(
            t=t, ranks=list(orc.ranks), eps=rec["eps"],
            e_over_eps=[e / rec["eps"] for e in rec["e_norm"]], q_over_eps=rec["q"] / rec["eps"],
            grew=[int(g) for g in rec["r_new"]], ignored=bool(rec["ignored"]),
            bound=orc.recon_error_bound()))
        if t in checkpoints:
            probes = []
            for tp in sorted({0, t // 2, t}):
                d = flat32(tp)
                probes.append(dict(t=tp, recon=vec(orc.reconstruct_slice(tp))[pos].tolist(),
                                   data=d[pos].tolist(), slice_norm=float(np.linalg.norm(d))))
            out["checkpoints"].append(dict(after=t, probes=probes))
        print(t, orc.ranks, f"{time.time() - t0:.0f}s", flush=True)
    name = ("fourier512_oracle_trajectory.json" if core_update == "literal"
            else f"fourier512_oracle_trajectory_{core_update}.json")
    # how far the auxiliary V of the core factorization is from orthonormal
    # (the Gram-based SVD of Alg. 1 leaves about u (s_1 / s_r)^2)
    vm = orc.vmat()
    out["final_v_orth"] = float(np.max(np.abs(vm.T @ vm - np.eye(vm.shape[1]))))
    out["init_v_orth"] = init_v_orth
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
