"""Host-side parts of the benchmark: the one-GPU refusal and the CPU-baseline leg (the oracle timed on a sample)."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_cpu_baseline_record():
    scene, cam = sg.make_small_terrain(seed=4, grid=16, n_spheres=2, level=1, lights=2, depth=2)
    cam = cam.resized(40, 30)
    rays_per_frame = 5000
    base, orc = bench.cpu_baseline(scene, cam, rays_per_frame, target_s=0.5)
    assert base["kind"] == "oracle" and base["unit"] == "Mrays/s" and base["value"] > 0
    assert base["cores"] >= 1 and base["paths"] == len(orc["samples"]) and base["rays"] == int(orc["ray_counts"].sum())
    assert base["one_thread"]["value"] > 0
    assert np.isclose(base["frame_seconds"], rays_per_frame / (base["value"] * 1e6))
    h = base["hierarchy_mode"]
    # the tree mode answers the brute-force sample identically, and is timed without its tree build
    assert h["identical_to_brute_force_on_sample"] is True
    assert h["value"] > 0 and h["trace_seconds"] > 0 and h["tree_build_seconds"] >= 0
    assert h["paths"] == base["paths"] + min(2 * cam.width * cam.height, 1 << 18)
