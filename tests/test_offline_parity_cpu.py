"""The two-step large-sample parity script on a small scene: the oracle step (chunked and resumable) and the
comparison (input digests, sample alignment, ties).  The stand-in GPU files here are written from the oracle's
own result, so they check the script's plumbing, not a GPU."""
import argparse
import os

import numpy as np
import pytest

import scenegen as sg
from tests import offline_parity as op


def _oracle(tmp, paths, chunk=64, seed=3):
    out = os.path.join(tmp, "orc.npz")
    op.run_oracle(argparse.Namespace(workload="spheres8_256", paths=paths, seed=seed, threads=2, chunk=chunk, out=out))
    return out


def _gpu_file(tmp, orc_path, name="gpu.npz", mutate=None, digest=None):
    o = np.load(orc_path)
    g = {k: o[k].copy() for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state")}
    g["radiance"] = g["radiance"].astype(np.float32)
    g["hit_t"] = g["hit_t"].astype(np.float32)
    if mutate:
        mutate(g)
    path = os.path.join(tmp, name)
    np.savez(path, digest=digest if digest is not None else str(o["digest"]), samples=o["samples"], **g)
    return path


def test_oracle_step_is_chunked_and_resumable(tmp_path, capsys):
    tmp = str(tmp_path)
    full = _oracle(tmp, 300, chunk=300)
    whole = dict(np.load(full))
    os.remove(full)
    # an interrupted run left the first 64 paths of the same sample
    np.savez(full + ".part.npz", digest=whole["digest"], samples=whole["samples"][:64],
             **{k: whole[k][:64] for k in op.FIELDS}, ray_counts=np.zeros(3, np.int64))
    capsys.readouterr()
    resumed = _oracle(tmp, 300, chunk=64)
    assert "64 already done" in capsys.readouterr().out
    z = np.load(resumed)
    assert np.array_equal(z["samples"], whole["samples"])
    for k in op.FIELDS:
        assert np.array_equal(z[k], whole[k]), k
    assert not os.path.exists(full + ".part.npz")
    scene, cam = sg.make_spheres_scene()
    assert str(z["digest"]) == sg.digest(scene, cam)


def test_compare_counts_ties_and_refuses_mismatched_inputs(tmp_path):
    tmp = str(tmp_path)
    orc = _oracle(tmp, 256)
    same = _gpu_file(tmp, orc)
    s = op.run_compare(argparse.Namespace(oracle=orc, gpu=same))
    assert s["passed"] and s["ties"] == 0 and s["n"] == 256 and s["max_err"] < 1e-6
    o = np.load(orc)
    hit = int(np.nonzero(o["path_prims"][:, 0] >= 0)[0][0])

    def wrong_primitive(g):  # a hit id the oracle does not certify: a real mismatch
        g["path_prims"][hit, 0] = (g["path_prims"][hit, 0] + 1) % 9
    bad = _gpu_file(tmp, orc, "bad.npz", mutate=wrong_primitive)
    s = op.run_compare(argparse.Namespace(oracle=orc, gpu=bad, details=True))
    assert s["ties"] == 1 and not s["passed"] and s["tie_ids"] == [int(o["samples"][hit])]
    assert s["tie_details"] == [{"path": int(o["samples"][hit]), "depth": 0, "kind": "hit",
                                 "oracle": int(o["path_prims"][hit, 0]),
                                 "gpu": int((o["path_prims"][hit, 0] + 1) % 9),
                                 "margin": float(o["hit_margin"][hit, 0])}]
    assert s["uncertified"] and s["uncertified"][0][0] == int(o["samples"][hit])

    def brighter(g):
        g["radiance"][hit] += 2e-4
    s = op.run_compare(argparse.Namespace(oracle=orc, gpu=_gpu_file(tmp, orc, "b.npz", mutate=brighter)))
    assert not s["passed"] and s["max_err"] > 1e-4
    with pytest.raises(SystemExit):
        op.run_compare(argparse.Namespace(oracle=orc, gpu=_gpu_file(tmp, orc, "d.npz", digest="0" * 64)))
