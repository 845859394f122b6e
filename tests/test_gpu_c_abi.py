"""The C ABI from plain C: tests/c_abi/query_main.c (built by
__graft_entry__.build()) links libtpa.so and the HIP runtime, builds the
rmat13 graph, preprocesses it and runs a batched query and single-seed
queries through include/tpa.h with hipMalloc'd buffers.  Its outputs must
match the FP64 oracle (L1 <= 1e-5 per seed), with no Python binding or torch
on the path."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import tpa_inputs as ti

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c_abi", "query_main")
c, S, T, EPS = ti.C, ti.S, ti.T, ti.EPS


def test_plain_c_caller_matches_oracle(tmp_path):
    assert os.path.exists(EXE), f"{EXE} is missing: run __graft_entry__.build()"
    scale, samples, seed = ti.GRAPHS["rmat13"]
    og = oracle.Graph.rmat(scale, samples, seed)
    og.preprocess(c, T, EPS)
    seeds = [int(s) for s in ti.draw_seeds(og.export()["padded"] == 0, 5, 77)]
    out = tmp_path / "r.bin"
    print("c abi caller: rmat13, seeds", seeds, flush=True)
    res = subprocess.run([EXE, str(scale), str(samples), str(seed), repr(c), str(S), str(T), str(out),
                          *map(str, seeds)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert f"n={og.n} m={og.m} k={len(seeds)}" in res.stdout
    R = np.fromfile(out, np.float32).reshape(2, len(seeds), og.n).astype(np.float64)
    for j, s in enumerate(seeds):
        expect = og.query(s, c, S, T)
        assert np.abs(R[0, j] - expect).sum() <= 1e-5, (s, "batched")
        assert np.abs(R[1, j] - expect).sum() <= 1e-5, (s, "single")
