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
    assert L.aco_strerror(-99) == b"ACO_ERR_UNKNOWN"
    assert b"gfx950" in L.aco_version()


def test_workspace_queries(L):
    n, k, m = 20000, 16, 256
    assert L.aco_construct_workspace_bytes(n, k) == n * k * 8
    assert L.aco_update_workspace_bytes(n, k, m) >= n * k * 8 + m * 8
    g = L.aco_grid_bytes(n)
    assert g >= 16 * n + 4 * (3 * n + 3)
    p = aco.AcoParams(m=m, k=k, alpha=1.0, beta=2.0, rho=0.1, iterations=50, deposit_shift=32,
                      seed=2)
    total = L.aco_run_workspace_bytes(n, C.byref(p))
    assert total >= m * n * 5 + n * k * (4 + 4 + 1 + 4 + 4 + 8 + 8) + g
    assert L.aco_grid_bytes(0) == 0


def test_validation_before_any_device_call(L):
    # every call below fails validation on the host; NULL pointers are never touched
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
    # windowed 2-opt: window, p, batch, round cap and NULL arrays, all before the GPU
    st = aco.AcoTwoOptStats()
    for window, p, batch, rounds in ((0, 0.5, 1, 0), (2049, 0.5, 1, 0), (10, 1.5, 1, 0),
                                     (10, float("nan"), 1, 0), (10, 0.5, 0, 0), (10, 0.5, 1, -1),
                                     (10, 0.5, 1, 0)):
        assert L.aco_two_opt(None, 100, 4, None, None, None, window, p, 1, 0, rounds, batch,
                             C.byref(st), None, 0, None) == aco.ACO_ERR_INVALID_ARG
    assert L.aco_two_opt_workspace_bytes(200000, 1024, 8) >= 8 * 200000 * 8
    assert L.aco_two_opt_workspace_bytes(0, 1, 1) == 0


def test_no_oracle_in_product_path():
    # the product package never imports, links or reads the oracle
    pkg = os.path.join(ROOT, "paper_1709_03187_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "instances.py", f
