"""The C-ABI library loads and exports every symbol include/aco.h declares;
host-side queries and argument validation work without a GPU (validation
happens before anything is enqueued, so no device call is made)."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_1709_03187_amd as aco

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aco.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aco_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(aco.LIB_PATH):
        pytest.skip("libaco.so not built")
    return aco.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("aco_build_candidates", "aco_construct_tours", "aco_update_pheromone",
                     "aco_run"):
        assert required in names
    assert set(names) == set(aco.EXPORTS)


def test_every_declared_symbol_is_exported(L):
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", aco.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (aco_[a-z0-9_]+)", out))
    assert set(declared_functions()) <= exported


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "aco.h"\nint main(void){ aco_params_t p; (void)p; return 0; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                    "-c", str(src), "-o", str(tmp_path / "t.o")], check=True)


def test_strerror_and_version(L):
    assert L.aco_strerror(0) == b"ACO_OK"
    assert L.aco_strerror(-1) == b"ACO_ERR_INVALID_ARG"
    assert L.aco_strerror(-4) == b"ACO_ERR_WORKSPACE"
    assert L.aco_strerror(-6) == b"ACO_ERR_DEVICE"
    assert L.aco_strerror(-99) == b"ACO_ERR_UNKNOWN"
    assert b"gfx950" in L.aco_version()


def test_workspace_queries(L):
    n, k, m = 20000, 16, 256
    assert L.aco_construct_workspace_bytes(n, k) == n * k * 8
    # rows start on 128-byte lines: 16, 32 or 64 elements of 8 bytes
    assert L.aco_construct_workspace_bytes(n, 5) == n * 16 * 8
    assert L.aco_construct_workspace_bytes(n, 12) == n * 16 * 8
    assert L.aco_construct_workspace_bytes(n, 17) == n * 32 * 8
    assert L.aco_construct_workspace_bytes(n, 40) == n * 64 * 8
    assert L.aco_update_workspace_bytes(n, k, m) >= n * k * 8 + m * 8
    g = L.aco_grid_bytes(n)
    assert g >= 16 * n + 4 * (3 * n + 3)
    p = aco.AcoParams(m=m, k=k, alpha=1.0, beta=2.0, rho=0.1, iterations=50, deposit_shift=32,
                      seed=2)
    total = L.aco_run_workspace_bytes(n, C.byref(p))
    assert total >= m * n * 5 + n * k * (4 + 4 + 1 + 4 + 4 + 8 + 8) + g
    assert L.aco_grid_bytes(0) == 0
    # the one query by kind agrees with each entry point's own
    W = aco.aco_workspace_bytes
    assert W(aco.ACO_WS_GRID, n, k, m) == g
    assert W(aco.ACO_WS_CONSTRUCT, n, k, m) == L.aco_construct_workspace_bytes(n, k)
    assert W(aco.ACO_WS_UPDATE, n, k, m) == L.aco_update_workspace_bytes(n, k, m)
    assert W(aco.ACO_WS_RUN, n, k, m) == total
    assert W(aco.ACO_WS_TWO_OPT, n, k, m) == L.aco_two_opt_workspace_bytes(n, m, 1)
    assert W(aco.ACO_WS_FEATURES, n, k, m) == L.aco_features_workspace_bytes()
    assert W(aco.ACO_WS_MLP_BACKWARD, n, k, m) == L.aco_mlp_backward_workspace_bytes(n * k)
    assert W(99, n, k, m) == 0
    # the learned heuristic adds the features (32 bytes per slot) and their workspace
    pl = aco.AcoParams(m=m, k=k, alpha=1.0, beta=2.0, rho=0.1, iterations=50, deposit_shift=32,
                       seed=2, eta_mode=aco.ACO_ETA_LEARNED)
    assert L.aco_run_workspace_bytes(n, C.byref(pl)) >= total + 32 * n * k
    # parameters: struct_size must cover the fields through seed
    assert p.struct_size == C.sizeof(aco.AcoParams)
    short = aco.AcoParams(m=m, k=k, alpha=1.0, beta=2.0, rho=0.1, iterations=50,
                          deposit_shift=32, seed=2)
    short.struct_size = 24
    assert L.aco_run_workspace_bytes(n, C.byref(short)) == 0
    # a caller built before eta_mode existed: its fields are read, the rest default
    short.struct_size = aco.AcoParams.seed.offset + 8
    short.eta_mode = 7            # beyond struct_size: never read
    assert L.aco_run_workspace_bytes(n, C.byref(short)) == total


def test_validation_before_any_device_call(L):
    # every call below fails validation on the host; NULL pointers are never touched,
    # nor the fake non-NULL one
    fake = C.c_void_p(16)
    assert L.aco_build_candidates(None, 2, 1, 2.0, None, None, None, None, None, None, 0,
                                  None) == aco.ACO_ERR_INVALID_ARG
    assert b"n = 2" in L.aco_last_error()
    assert L.aco_build_candidates(None, 100, 0, 2.0, None, None, None, None, None, None, 0,
                                  None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_build_candidates(None, 100, 65, 2.0, None, None, None, None, None, None, 0,
                                  None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_build_candidates(None, 100, 8, -1.0, None, None, None, None, None, None, 0,
                                  None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_build_candidates(None, 100, 8, 2.0, None, None, None, None, None, None, 0,
                                  None) == aco.ACO_ERR_INVALID_ARG   # NULL arrays
    assert L.aco_construct_tours(None, 100, 8, None, None, None, None, None, 0, 0, 1.0, 1, 0,
                                 None, None, None, None, None, 0, None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_construct_tours(None, 100, 8, None, None, None, None, None, 4, 0, float("nan"),
                                 1, 0, None, None, None, None, None, 0,
                                 None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_update_pheromone(100, 8, None, None, 4, None, None, None, 0.0, 32, None, None, 0,
                                  None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_update_pheromone(100, 8, None, None, 4, None, None, None, 0.1, 63, None, None, 0,
                                  None) == aco.ACO_ERR_INVALID_ARG
    p = aco.AcoParams(m=0, k=8, alpha=1.0, beta=2.0, rho=0.1, iterations=1, deposit_shift=32,
                      seed=1)
    assert L.aco_run(None, 100, C.byref(p), None, None, None, None, None, 0,
                     None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_run(None, 100, None, None, None, None, None, None, 0,
                     None) == aco.ACO_ERR_INVALID_ARG
    for mode, w in ((5, None), (aco.ACO_ETA_LEARNED, None)):
        p = aco.AcoParams(m=4, k=8, alpha=1.0, beta=2.0, rho=0.1, iterations=1, deposit_shift=32,
                          seed=1, eta_mode=mode, mlp_w=w)
        assert L.aco_run(None, 100, C.byref(p), None, None, None, None, None, 0,
                         None) == aco.ACO_ERR_INVALID_ARG
        assert b"eta_mode" in L.aco_last_error() or b"mlp_w" in L.aco_last_error()
    p.struct_size = 16
    assert L.aco_run(None, 100, C.byref(p), None, None, None, None, None, 0,
                     None) == aco.ACO_ERR_INVALID_ARG
    assert b"struct_size" in L.aco_last_error()
    # batched colonies: eta = 1/d only; k = 0 is for aco_run_batched alone
    off = (C.c_int64 * 3)(0, 50, 120)
    p = aco.AcoParams(m=4, k=8, alpha=1.0, beta=2.0, rho=0.1, iterations=1, deposit_shift=32,
                      seed=1, eta_mode=aco.ACO_ETA_LEARNED, mlp_w=16)
    assert L.aco_batch_setup(fake, off, 2, C.byref(p), fake, fake, fake, 1 << 30,
                             None) == aco.ACO_ERR_UNSUPPORTED
    p = aco.AcoParams(m=4, k=0, alpha=1.0, beta=2.0, rho=0.1, iterations=1, deposit_shift=32,
                      seed=1)
    assert L.aco_batch_setup(fake, off, 2, C.byref(p), fake, fake, fake, 1 << 30,
                             None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_batch_workspace_bytes(off, 2, C.byref(p)) == L.aco_batch_workspace_bytes(
        off, 2, C.byref(aco.AcoParams(m=4, k=16, alpha=1.0, beta=2.0, rho=0.1, iterations=1,
                                      deposit_shift=32, seed=1)))
    # windowed 2-opt: window, p, batch, round cap and NULL arrays, all before the GPU
    st = aco.AcoTwoOptStats()
    for window, p, batch, rounds in ((0, 0.5, 1, 0), (2049, 0.5, 1, 0), (10, 1.5, 1, 0),
                                     (10, float("nan"), 1, 0), (10, 0.5, 0, 0), (10, 0.5, 1, -1),
                                     (10, 0.5, 1, 0)):
        assert L.aco_two_opt(None, 100, 4, None, None, None, window, p, 1, 0, rounds, batch,
                             C.byref(st), None, 0, None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_two_opt_workspace_bytes(200000, 1024, 8) >= 8 * 200000 * 8
    assert L.aco_two_opt_workspace_bytes(0, 1, 1) == 0
    # local-best pheromone: m * 2^shift must stay below 2^63 (checked before the arrays)
    assert L.aco_pheromone_local_best(100, 8, fake, fake, 1024, fake, fake, 1.0, 1.0, 53, fake,
                                      fake, 1 << 30, None) == aco.ACO_ERR_INVALID_ARG
    assert b"overflow" in L.aco_last_error()
    assert L.aco_pheromone_local_best(100, 8, None, None, 1024, None, None, 1.0, 1.0, 52, None,
                                      None, 0, None) == aco.ACO_ERR_INVALID_ARG
    assert b"NULL" in L.aco_last_error()
    # construction options: struct_size must cover the fields through lbest
    opts = aco.AcoConstructOpts(aco.ACO_SAMPLER_ROULETTE, 0.0, 1, None, None)
    assert opts.struct_size == C.sizeof(aco.AcoConstructOpts)
    opts.struct_size = 8
    assert L.aco_construct_ex(fake, 100, 8, fake, fake, fake, fake, fake, 4, 0, 1.0, 1, 0,
                              C.byref(opts), fake, fake, fake, None, fake, 1 << 30,
                              None) == aco.ACO_ERR_INVALID_ARG
    assert b"struct_size" in L.aco_last_error()


def test_no_oracle_in_product_path():
    # the product package never imports, links or reads the oracle
    pkg = os.path.join(ROOT, "paper_1709_03187_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "instances.py", f
