"""C-ABI library: exports, validation and the host-side setup tables (no GPU use).

The host tables are compared with the oracle's independent dense construction
(T. Chan columns by the closed form, eigenvalues by explicit DFT sums)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import grunwald, precond
from oracle import operator as op
from paper_1907_13428_amd import fde

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(fde.LIB_PATH), reason="libfde.so not built")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fde.h")).read()
    return sorted(set(re.findall(r"\b(fde_[a-z_A-Z]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = fde.lib()
    names = declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(fde.EXPORTED) == set(names)


def test_version_and_empty_error():
    assert b"gfx950" in fde.lib().fde_version()


@pytest.mark.parametrize("field,value,frag", [
    ("nx", 10, "nx=10"), ("ny", 2, "ny=2"), ("nt", 2048, "nt=2048"), ("alpha", 1.0, "alpha"),
    ("beta", 2.5, "beta"), ("T", 0.0, "T must"), ("ctrl_sign", 0.5, "ctrl_sign"),
    ("obj_weights", 3, "obj_weights"), ("precond_fp32", 2, "precond_fp32")])
def test_problem_validation(field, value, frag):
    w = W.small()
    prob, prm = fde.from_workload(w)
    setattr(prob, field, value)
    with pytest.raises(fde.FdeError) as e:
        fde.validate(prob, prm)
    assert e.value.status == fde.FDE_EINVAL and frag in str(e.value)


@pytest.mark.parametrize("field,value", [("gamma", 0.0), ("delta", -1.0), ("rho", 1.7), ("rho", 0.0),
                                         ("krylov_maxit", 0), ("admm_maxit", 0), ("tol_mode", 5),
                                         ("ya", 1.0), ("ua", math.nan), ("krylov_tol", -1.0),
                                         ("precond_kind", 3), ("precond_kind", -1), ("krylov_solver", 2)])
def test_param_validation(field, value):
    w = W.small()
    prob, prm = fde.from_workload(w)
    if field == "ya":
        prm.yb = 0.0
    setattr(prm, field, value)
    with pytest.raises(fde.FdeError):
        fde.validate(prob, prm)


def test_negative_coefficient_rejected():
    w = W.small()
    w.dplus = -np.ones((w.ny, w.nx))
    prob, prm = fde.from_workload(w)
    with pytest.raises(fde.FdeError):
        fde.validate(prob, prm)


def test_supported_sizes():
    w = W.small()
    for n in (4, 6, 8, 12, 16, 24, 48, 50, 80, 96, 100, 160, 192, 256, 384, 512, 768, 1024):
        prob, prm = fde.from_workload(w.replace(nx=n, ny=n, nt=n, yhat=None))
        fde.validate(prob, prm)
    for n in (3, 5, 9, 10, 18, 20, 36, 40, 200, 1536, 2048):
        prob, prm = fde.from_workload(w.replace(nx=n, yhat=None))
        with pytest.raises(fde.FdeError):
            fde.validate(prob, prm)


@pytest.mark.parametrize("wl", ["small", "headline_small", "trap", "caputo", "paper_16", "prox", "prox_default"])
def test_host_tables_match_oracle(wl):
    if wl == "small":
        w = W.small()
    elif wl == "headline_small":
        w = W.headline(nx=24, ny=16, nt=8)
    elif wl == "caputo":
        w = W.small_mixed(nx=12, ny=8, nt=6, alpha_t=0.4, T=0.7)
    elif wl == "paper_16":
        w = W.paper_test(16)
    elif wl == "prox":
        w = W.small_mixed(nx=12, ny=8, nt=6, obj_weights=1, rho=0.8, delta=0.4, prox=1, prox_cy=1.7, prox_cu=3e-3)
    elif wl == "prox_default":
        w = W.small_mixed(nx=12, ny=8, nt=6, obj_weights=1, prox=1)
    else:
        w = W.small_mixed(nx=12, ny=8, nt=6, obj_weights=1, rho=1.618, delta=0.4)
    prob, prm = fde.from_workload(w)
    t = fde.host_tables(prob, prm)
    d = op.disc_from(w)
    tab = precond.precond_tables(w, d)
    assert t["psi"] == pytest.approx(tab["psi"], rel=1e-15)
    assert t["a"] == pytest.approx(tab["a"], rel=1e-14)
    assert t["inv_mbar"] == pytest.approx(1.0 / tab["mbar_p"], rel=1e-14)
    assert t["hx"] == d.hx and t["hy"] == d.hy and t["ht"] == pytest.approx(d.ht, rel=1e-15)
    for k in ("lam_x", "lam_y", "lam_t"):
        ref = tab[k]
        assert np.max(np.abs(t[k] - ref)) <= 1e-12 * np.max(np.abs(ref)), k
    np.testing.assert_allclose(t["gx"], grunwald.weights(w.alpha, w.nx), rtol=1e-15, atol=1e-300)
    np.testing.assert_allclose(t["gy"], grunwald.weights(w.beta, w.ny), rtol=1e-15, atol=1e-300)


@pytest.mark.parametrize("bad", [-0.5, 1.5, float("nan")])
def test_time_order_validation(bad):
    prob, prm = fde.from_workload(W.small().replace(alpha_t=bad))
    with pytest.raises(fde.FdeError) as e:
        fde.validate(prob, prm)
    assert e.value.status == fde.FDE_EINVAL and "alpha_t" in str(e.value)


@pytest.mark.parametrize("field,value,frag", [("prox", 2, "prox must"), ("rho", 1.2, "rho in (0, 1]"),
                                              ("prox_cy", 0.5, "prox_cy"), ("prox_cy", -1.0, "prox_cy"),
                                              ("prox_cy", math.inf, "prox_cy"), ("prox_cu", 0.5e-4, "prox_cu"),
                                              ("prox_cu", math.nan, "prox_cu")])
def test_generalized_admm_validation(field, value, frag):
    """Algorithm 2: step in (0, 1]; R_y = c_y I - J1 and R_u = c_u I - J2 not
    indefinite (c_y >= 1, c_u >= gamma, or 0 for those values)."""
    w = W.small(prox=1)  # gamma = 1e-4
    prob, prm = fde.from_workload(w)
    fde.validate(prob, prm)
    setattr(prm, field, value)
    with pytest.raises(fde.FdeError) as e:
        fde.validate(prob, prm)
    assert e.value.status == fde.FDE_EINVAL and frag in str(e.value)
    # the same values are ignored under Algorithm 1 (rho up to the golden ratio)
    if field != "prox":
        prm.prox = 0
        fde.validate(prob, prm)


def test_time_order_zero_reads_as_implicit_euler():
    w = W.small()
    p0, prm = fde.from_workload(w.replace(alpha_t=0.0))
    p1, _ = fde.from_workload(w)
    t0, t1 = fde.host_tables(p0, prm), fde.host_tables(p1, prm)
    assert t0["psi"] == t1["psi"] and np.array_equal(t0["lam_t"], t1["lam_t"])


def test_product_path_has_no_cpu_fallback():
    """The binding refuses to run without a GPU instead of falling back."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    w = W.small()
    prob, prm = fde.from_workload(w)
    with pytest.raises(RuntimeError):
        fde.Context(prob, prm)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of fde_problem, fde_admm_params and fde_admm_stats
    have the C header's sizes and field offsets (compiled with the host C
    compiler)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"fde_problem": fde.Problem, "fde_admm_params": fde.Params, "fde_admm_stats": fde.Stats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "fde.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        cname, field, val = line.split()
        cls = structs[cname]
        want = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(val) == want, (cname, field, int(val), want)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())


@pytest.mark.parametrize("alpha_t", [1.0, 0.6])
def test_host_diag_scaling_matches_oracle(alpha_t):
    """fde_host_diag_scaling (the C++ setup of precond_kind 2) against the
    oracle's Delta = (s0 / diag S)^{1/2} from the assembled D."""
    from oracle import admm
    from oracle import precond as pc

    w = W.small(nx=12, ny=8, nt=6).replace(obj_weights=1, alpha_t=alpha_t, precond_kind=2)
    rng = np.random.Generator(np.random.PCG64(4))
    w.dplus = 0.5 + rng.uniform(size=(w.ny, w.nx))
    w.dminus = 0.3 + rng.uniform(size=(w.ny, w.nx))
    prob, prm = fde.from_workload(w)
    got = fde.host_diag_scaling(prob, prm)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    want = pc.scaling_factor(pc.diag_S(w, d, sc.My, sc.Mp, sc.psi))
    np.testing.assert_allclose(got, want, rtol=1e-12)
    # precond_kind 2 is a PCG preconditioner: MINRES with it is rejected
    _, prm2 = fde.from_workload(w.replace(krylov_solver=1))
    assert lib_validate(prob, prm2) == fde.FDE_EINVAL


def lib_validate(prob, prm):
    return fde.lib().fde_validate(ctypes.byref(prob), ctypes.byref(prm))
