"""The on-disk cache of tuned transform tiles: a context's tuning of a batched float32 shape is
written to the cache file and a new context starts with it; lines of another device or
version, and unreadable lines, are ignored; an empty path disables the cache."""
import numpy as np
import pytest

from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import make_problem, oracle_data

pytestmark = pytest.mark.gpu


def _probs(lib, torch, n=64, k=5):
    wls = [WL.shear_workload(n, 300 + i, nbands_e=3, nbands_b=3) for i in range(k)]
    return [make_problem(lib, torch, wl, "f32", d=oracle_data(wl, 310 + i)) for i, wl in enumerate(wls)]


def test_tuned_tiles_persist_across_contexts(lib, tmp_path, monkeypatch):
    import torch
    print("[tune cache]", flush=True)
    path = tmp_path / "sub" / "tiles.txt"
    monkeypatch.setenv("WF_TUNE_CACHE", str(path))
    probs = _probs(lib, torch)
    cx = lib.Context(0)
    try:
        assert lib.get_chain_tiles(64, 2, lib.WF_F32, 5, ctx=cx)[4] is False
        s1, _, st1, _ = lib.map_wf_solve(probs, lib.LbfgsOpts(rel_grad_tol=1e-6), ctx=cx)
        tuned = lib.get_chain_tiles(64, 2, lib.WF_F32, 5, ctx=cx)
        assert tuned[4] is True
    finally:
        cx.close()
    lines = path.read_text().split("\n")
    fields = [l.split() for l in lines if l.strip()]
    assert any(f[2:6] == ["64", "2", "0", "4"] and [int(x) for x in f[6:10]] == list(tuned[:4]) for f in fields)
    dev = fields[0][1]
    # a new context starts from the file: the same choice, and the same fields bit for bit
    cx2 = lib.Context(0)
    try:
        assert lib.get_chain_tiles(64, 2, lib.WF_F32, 5, ctx=cx2) == tuned
        s2, _, st2, _ = lib.map_wf_solve(probs, lib.LbfgsOpts(rel_grad_tol=1e-6), ctx=cx2)
        assert all(torch.equal(a, b) for a, b in zip(s1, s2))
    finally:
        cx2.close()
    # another device or version, and garbage, are ignored
    path.write_text(f"0 {dev} 64 2 0 4 2 1 0 0\n1 other/1 64 2 0 4 2 1 0 0\nnot a line\n")
    cx3 = lib.Context(0)
    try:
        assert lib.get_chain_tiles(64, 2, lib.WF_F32, 5, ctx=cx3)[4] is False
    finally:
        cx3.close()
    # an empty path: no cache read or written
    off = tmp_path / "off.txt"
    monkeypatch.setenv("WF_TUNE_CACHE", "")
    cx4 = lib.Context(0)
    try:
        lib.map_wf_solve(probs, lib.LbfgsOpts(rel_grad_tol=1e-6), ctx=cx4)
        assert lib.get_chain_tiles(64, 2, lib.WF_F32, 5, ctx=cx4)[4] is True
    finally:
        cx4.close()
    assert not off.exists()
    assert np.isfinite(st1[0].chi2)
