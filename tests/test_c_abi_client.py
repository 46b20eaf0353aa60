"""The plain C client of the ABI (paper_1907_13428_amd/examples/c_abi_demo.c):
no Python binding and no PyTorch between it and libfde.so.  On the CPU it
must reject an invalid problem through fde_validate; on the GPU its operator,
preconditioner and PCG results must match the oracle."""
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import admm, precond
from oracle import operator as op

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "paper_1907_13428_amd", "examples", "c_abi_demo")


def binary():
    if not os.path.exists(BIN):
        pytest.fail("examples/c_abi_demo is not built (run __graft_entry__.build())")
    return BIN


def test_c_client_rejects_an_invalid_problem(tmp_path):
    r = subprocess.run([binary(), "10", "8", "4", "1.5", "1.5", str(tmp_path / "o.bin")], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 1
    assert "fde_validate" in r.stderr and "nx=10" in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("shape,orders", [((24, 16, 8), (1.5, 1.3)), ((48, 12, 6), (1.8, 1.2))])
def test_c_client_matches_oracle(tmp_path, shape, orders):
    nx, ny, nt = shape
    a, b = orders
    print(f"[case] C client {nx}x{ny}x{nt} orders {a}/{b}", flush=True)
    out = tmp_path / "o.bin"
    r = subprocess.run([binary(), str(nx), str(ny), str(nt), repr(a), repr(b), str(out)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    n = nx * ny * nt
    got = np.fromfile(out, dtype=np.float64).reshape(4, nt, ny, nx)
    x = (((37 * np.arange(n, dtype=np.int64)) % 101) / 101.0 - 0.5).reshape(nt, ny, nx)
    w = W.Workload(name="c_client", nx=nx, ny=ny, nt=nt, alpha=a, beta=b, gamma=1e-4, ua=-1.0, ub=1.0)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = precond.precond_tables(w, d)

    def rel(u, v):
        return float(np.linalg.norm(u - v) / np.linalg.norm(v))

    assert rel(got[0], op.apply_D(d, x)) <= 1e-11
    assert rel(got[1], op.apply_DT(d, x)) <= 1e-11
    assert rel(got[2], precond.apply_precond(tab, x)) <= 1e-11
    ref, itr, _, conv = admm.pcg(lambda v: admm.apply_S(d, sc, v), lambda v: precond.apply_precond(tab, v), x,
                                 np.zeros(w.shape), 1e-10, 1000)
    it = int(re.search(r"pcg_iters=(\d+)", r.stdout).group(1))
    assert conv and abs(it - itr) <= 1
    assert rel(got[3], ref) <= 1e-9
