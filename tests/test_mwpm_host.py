"""The library's matching solver (its own source, mwpm_solver.h, built for the
host with one lane and run under the address and undefined-behaviour
sanitizers) against the oracle's exact matching parts, problem by problem,
before any of it runs on a GPU.  Bit-exact: every (type, parity) part of
every syndrome, at every size including fully lit syndromes.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import geometry, sampler
from oracle import matching as mm

from paper_1302_2669_amd.inputs import uniform_syndromes

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def host_solver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path_factory.mktemp("mwpm") / "mwpm_host")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe,
           os.path.join(HERE, "mwpm_host.cpp")]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def run_host(exe, L, syn):
    syn = np.ascontiguousarray(syn, dtype=np.uint8)
    n = syn.shape[0]
    data = np.array([L, n], dtype=np.int32).tobytes() + syn.tobytes()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    res = subprocess.run([exe], input=data, capture_output=True, env=env, timeout=600)
    assert res.returncode == 0, res.stderr.decode()[-3000:]
    rows = 2 * L - 1
    out = np.frombuffer(res.stdout, dtype=np.uint32).reshape(n, 4, 1 + rows)
    return out[:, :, 0].astype(bool), out[:, :, 1:]


def oracle_rows(lat, part):
    """Bit rows (bit f of row r = field f of grid row r) of a per-qubit part."""
    rows = np.zeros(2 * lat.L - 1, dtype=np.uint32)
    for q in np.nonzero(part)[0]:
        r, c = (int(v) for v in lat.qubit_rc[q])
        rows[r] |= np.uint32(1 << (c >> 1))
    return rows


def check(exe, L, syn):
    lat = geometry.Lattice(L)
    failed, planes = run_host(exe, L, syn)
    assert not failed.any()
    for s in range(syn.shape[0]):
        for p in range(4):
            part, _ = mm.type_part(lat, syn[s], p >> 1 == 1, p & 1)
            assert np.array_equal(planes[s, p], oracle_rows(lat, part)), (L, s, p)


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 7, 9])
def test_host_solver_random_syndromes(host_solver, L):
    lat = geometry.Lattice(L)
    syn = np.concatenate([uniform_syndromes(L, 12, seed=300 + L, density=0.3),
                          uniform_syndromes(L, 12, seed=400 + L, density=0.1),
                          uniform_syndromes(L, 4, seed=500 + L, density=0.7),
                          np.zeros((1, lat.n_stab), np.uint8),
                          np.ones((1, lat.n_stab), np.uint8)])
    check(host_solver, L, syn)


@pytest.mark.parametrize("L,p,n", [(13, 0.15, 6), (13, 0.05, 4), (17, 0.16, 2)])
def test_host_solver_sampled_syndromes(host_solver, L, p, n):
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, 0x1302266900000013, np.arange(n))
    check(host_solver, L, syn)


def test_host_solver_largest_codes(host_solver):
    """L = 25 near threshold (about 200 matching vertices per problem, one
    wave per workgroup on the GPU) and a fully lit L = 17 syndrome (274)."""
    lat = geometry.Lattice(25)
    syn, _, _ = sampler.sample(lat, 0.18, 5, np.arange(1))
    check(host_solver, 25, syn)
    lat = geometry.Lattice(17)
    check(host_solver, 17, np.ones((1, lat.n_stab), np.uint8))
