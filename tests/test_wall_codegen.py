"""The generated no-slip wall arithmetic (csrc/mbs_wall_gen.h, written by
paper_1411_0278_amd/wall_codegen.py from Blake's image system in its own form) against the oracle's
wall blocks, on the CPU: the header is built for the host with g++ and evaluated pair by pair."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from oracle import wall  # noqa: E402

ETA, A = 1.0 / (6.0 * np.pi), 1.3
P = 1.0 / (8.0 * np.pi * ETA)


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("wallgen") / "wall_gen_host.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", out,
                    os.path.join(ROOT, "tests", "host", "wall_gen_host.cpp"),
                    "-I", os.path.join(ROOT, "paper_1411_0278_amd", "csrc")], check=True)
    return ctypes.CDLL(out)


def _p(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(ctypes.c_void_p)


def _pairs(n, seed):
    """Receivers above a wall at z = 0 against sources at heights >= a: R = x - y*, h = y_3."""
    rng = np.random.default_rng(seed)
    x = np.column_stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), rng.uniform(A, 9, n)])
    y = np.column_stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), rng.uniform(A, 9, n)])
    x[:4] = y[:4]  # a sphere and its own image
    R = x - y * np.array([1.0, 1.0, -1.0])
    geo = np.column_stack([R, y[:, 2], np.full(n, A * A), np.zeros(n)])
    return R, y[:, 2], geo, rng


def _close(got, want):
    return np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_generated_wall_operator_strain_matches_oracle(lib):
    n = 60
    R, h, geo, rng = _pairs(n, 1)
    sig = rng.standard_normal((n, 5))
    e = np.zeros((n, 5))
    lib.ev_strain_s(n, _p(geo), _p(P * sig), e.ctypes.data_as(ctypes.c_void_p))
    want = np.einsum("pij,pj->pi", wall.block("wall", "E", "S", R, h, A, ETA), sig)
    assert _close(e, want)


def test_generated_wall_rhs_strain_matches_oracle(lib):
    n = 60
    R, h, geo, rng = _pairs(n, 2)
    F, T, d = rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    e = np.zeros((n, 5))
    lib.ev_strain_ftq(n, _p(geo), _p(P * F), _p(P * T), _p(A ** 5 / 20 * d), e.ctypes.data_as(ctypes.c_void_p))
    want = sum(np.einsum("pij,pj->pi", wall.block("wall", "E", k, R, h, A, ETA), v)
               for k, v in (("F", F), ("T", T), ("D", d)))
    assert _close(e, want)


def test_generated_wall_motion_and_flow_match_oracle(lib):
    n = 60
    R, h, geo, rng = _pairs(n, 3)
    F, T, S, d = (rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), rng.standard_normal((n, 5)),
                  rng.standard_normal((n, 3)))
    args = [_p(P * F), _p(P * T), _p(P * S), _p(A ** 5 / 20 * d)]
    u, w, uf = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
    lib.ev_motion_ftsq(n, _p(geo), *args, u.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p))
    lib.ev_flow_ftsq(n, _p(geo), *args, uf.ctypes.data_as(ctypes.c_void_p))
    src = (("F", F), ("T", T), ("S", S), ("D", d))
    U = sum(np.einsum("pij,pj->pi", wall.block("wall", "U", k, R, h, A, ETA), v) for k, v in src)
    W = sum(np.einsum("pij,pj->pi", wall.block("wall", "W", k, R, h, A, ETA), v) for k, v in src)
    Uf = sum(np.einsum("pij,pj->pi", wall.flow("wall", k, R, h, A, ETA), v) for k, v in src)
    assert _close(u, U) and _close(w, W) and _close(uf, Uf)


def test_committed_header_is_what_the_generator_writes():
    from paper_1411_0278_amd import wall_codegen
    path = os.path.join(ROOT, "paper_1411_0278_amd", "csrc", "mbs_wall_gen.h")
    assert open(path).read() == wall_codegen.generate()
