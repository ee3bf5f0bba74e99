"""Large-sample parity between a GPU frame and the FP64 oracle, run outside pytest.

The oracle is too slow to cover a full 1080p stereo frame of the 3.4M-triangle scene inside a test
(every query tests every primitive), so the large sample is split in two steps that meet in files:

    # on a host: the oracle on a seeded sample of the frame's paths (resumable, chunk by chunk)
    python -m tests.offline_parity oracle --paths 131072 --seed 17 --out /tmp/orc_terrain3m_1080p.npz
    # on the GPU: the frame rendered once with ray-tree signatures, the same sample written out
    python bench.py --dump-signature /tmp/gpu_sig.npz --dump-paths 131072 --dump-seed 17 ...
    # anywhere: the comparison, with the tie rate and its 95% Clopper-Pearson upper bound
    python -m tests.offline_parity compare --oracle /tmp/orc_terrain3m_1080p.npz --gpu /tmp/gpu_sig.npz

The oracle step calls only the oracle and the seeded scene generator; the GPU file is never an input
to it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FIELDS = ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state", "hit_margin", "shadow_margin",
          "shadow_contrib")


def workload(name: str):
    import scenegen as sg
    if name == "terrain3.4M_1080p":
        return sg.make_terrain_3m()
    if name == "terrain3.4M_4k":
        s, c = sg.make_terrain_3m()
        return s, c.resized(3840, 2160)
    if name == "terrain212k_1080p":
        return sg.make_terrain_1080p()
    if name == "spheres8_256":
        return sg.make_spheres_scene()
    raise SystemExit(f"unknown workload {name}")


def run_oracle(args):
    import oracle
    import scenegen as sg
    scene, cam = workload(args.workload)
    digest = sg.digest(scene, cam)
    samples = sg.sample_paths(cam, args.paths, seed=args.seed)
    part = args.out + ".part.npz"
    done = {}
    if os.path.exists(part):
        z = np.load(part)
        if str(z["digest"]) == digest and np.array_equal(z["samples"], samples[:len(z["samples"])]):
            done = {k: z[k] for k in FIELDS}
            done["ray_counts"] = z["ray_counts"]
    n_done = len(done.get("hit_t", []))
    print(f"[oracle] {args.workload}: {len(samples)} paths (seed {args.seed}), {n_done} already done, "
          f"{args.threads} threads", flush=True)
    t_all = time.perf_counter()
    while n_done < len(samples):
        chunk = samples[n_done:n_done + args.chunk]
        t0 = time.perf_counter()
        r = oracle.render(scene, cam, samples=chunk, nthreads=args.threads)
        for k in FIELDS:
            done[k] = r[k] if k not in done else np.concatenate([done[k], r[k]])
        done["ray_counts"] = r["ray_counts"] + (done["ray_counts"] if "ray_counts" in done and n_done else 0)
        n_done += len(chunk)
        np.savez(part, digest=digest, samples=samples[:n_done], **done)
        print(f"[oracle] {n_done}/{len(samples)} paths ({time.perf_counter() - t0:.1f} s for {len(chunk)})",
              flush=True)
    np.savez(args.out, digest=digest, samples=samples, workload=args.workload, seed=args.seed,
             seconds=time.perf_counter() - t_all, threads=args.threads, **done)
    if os.path.exists(part):
        os.remove(part)
    print(f"[oracle] wrote {args.out}", flush=True)


def run_compare(args):
    from tests.parity import compare
    o = np.load(args.oracle)
    g = np.load(args.gpu)
    if str(o["digest"]) != str(g["digest"]):
        raise SystemExit("the oracle and GPU files were made from different inputs")
    if not np.array_equal(o["samples"], g["samples"]):
        raise SystemExit("the oracle and GPU files cover different paths")
    orc = {k: o[k] for k in FIELDS}
    orc["samples"] = np.arange(len(o["samples"]))  # the GPU arrays hold exactly the sampled paths
    gpu = {k: g[k] for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state")}
    res = compare(gpu, orc, allow_min_one=False)
    res["tie_ids"] = [int(o["samples"][i]) for i in res["tie_ids"]]
    res["uncertified"] = [(int(o["samples"][i]), m) for i, m in res["uncertified"]]
    if res["worst"] >= 0:
        res["worst"] = int(o["samples"][res["worst"]])
    summary = {"workload": str(o["workload"]), "seed": int(o["seed"]), "n": res["n"], "ties": res["ties"],
               "tie_rate": res["tie_rate"], "tie_rate_upper95": res["tie_rate_upper95"],
               "uncertified": res["uncertified"], "max_err": res["max_err"],
               "max_rel_t_err": res.get("max_rel_t_err"), "tie_ids": res["tie_ids"],
               "oracle_rays": int(np.asarray(o["ray_counts"]).sum()), "passed": res["passed"]}
    if getattr(args, "details", False):
        summary["tie_details"] = tie_details(gpu, orc, o["samples"])
    print(json.dumps(summary), flush=True)
    return summary


def tie_details(gpu: dict, orc: dict, samples) -> list:
    """For each tie path: the first decision where the GPU and the oracle differ, with the oracle's margin."""
    from tests.parity import CONTRIB_MIN, first_divergence
    prim = gpu["path_prims"] != orc["path_prims"]
    sh = (gpu["shadow_state"] != orc["shadow_state"]) & (orc["shadow_contrib"] > CONTRIB_MIN)
    tie = prim.any(axis=1) | sh.reshape(len(prim), -1).any(axis=1)
    out = []
    for k in np.nonzero(tie)[0]:
        kind, d, ls = first_divergence(prim[k], sh[k])
        if kind == "shadow":
            out.append({"path": int(samples[k]), "depth": d, "kind": "shadow", "lights": ls.tolist(),
                        "margin": float(orc["shadow_margin"][k, d, ls].min()),
                        "contribution": float(orc["shadow_contrib"][k, d, ls].max())})
        else:
            out.append({"path": int(samples[k]), "depth": d, "kind": "hit", "oracle": int(orc["path_prims"][k, d]),
                        "gpu": int(gpu["path_prims"][k, d]), "margin": float(orc["hit_margin"][k, d])})
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("oracle")
    a.add_argument("--workload", default="terrain3.4M_1080p")
    a.add_argument("--paths", type=int, default=1 << 17)
    a.add_argument("--seed", type=int, default=17)
    a.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a.add_argument("--chunk", type=int, default=4096)
    a.add_argument("--out", required=True)
    c = sub.add_parser("compare")
    c.add_argument("--oracle", required=True)
    c.add_argument("--gpu", required=True)
    c.add_argument("--details", action="store_true", help="list the first divergent decision of every tie")
    args = ap.parse_args()
    if args.cmd == "oracle":
        run_oracle(args)
    else:
        s = run_compare(args)
        sys.exit(0 if s["passed"] else 1)


if __name__ == "__main__":
    main()
