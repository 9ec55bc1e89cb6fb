"""Host-side checks of libmcmcdec: it loads, exports every symbol the header
declares, and its host-only entry points agree with the oracle.  No GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1302_2669_amd as mc
from paper_1302_2669_amd import _lib
from oracle import geometry, tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mcmcdec.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcmc_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = _lib._lib()
    decl = declared_symbols()
    assert decl == _lib.exported_symbols()
    for name in decl:
        assert hasattr(lib, name), name
    assert lib.mcmc_abi_version() == 0x00010000


@pytest.mark.parametrize("L", list(range(2, 26)))
def test_geometry_and_lattice_match_oracle(L):
    lat = geometry.Lattice(L)
    assert mc.geometry(L) == (lat.n_qubits, lat.n_stab)
    sup, col, drw = mc.lattice(L)
    for s in range(lat.n_stab):
        assert sorted(x for x in sup[s] if x >= 0) == sorted(lat.supports[s])
    assert np.array_equal(col, lat.site_colour)
    assert np.array_equal(drw, lat.draw_index)


@pytest.mark.parametrize("p", [0.01, 0.05, 0.1, 0.13, 0.15, 0.16, 0.17, 0.18, 0.3, 0.74])
@pytest.mark.parametrize("K", [1, 2, 20, 64])
def test_tables_match_oracle(p, K):
    assert np.array_equal(mc.acceptance_table(p, K), tables.tables(p, K))


def test_out_of_range_rejected():
    for L in (0, 1, 26, -3):
        with pytest.raises(mc.McmcError) as e:
            mc.geometry(L)
        assert e.value.status == -2
    for p in (0.0, 0.75, -1.0, float("nan"), 2.0):
        with pytest.raises(mc.McmcError):
            mc.acceptance_table(p)


def _ws(**kw):
    base = dict(L=9, p=0.1, sweeps=10, seed=1, chains=2, n_temps=1, burn=0)
    base.update(kw)
    return mc.workspace_size(mc.make_params(**base), 10)


@pytest.mark.parametrize("kw,status", [
    (dict(n_temps=3), -1), (dict(n_temps=0), -2), (dict(n_temps=66), -2),
    (dict(chains=0), -2), (dict(sweeps=-1), -2), (dict(burn=-2), -2),
    (dict(L=30), -2), (dict(p=0.8), -2), (dict(flags=8), -1), (dict(sweep_begin=3), -1),
    (dict(init=2), -1),
])
def test_param_validation(kw, status):
    with pytest.raises(mc.McmcError) as e:
        _ws(**kw)
    assert e.value.status == status


def test_decode_rejects_before_launch():
    """Bad arguments come back as status codes without touching a device."""
    lib = _lib._lib()
    prm = mc.make_params(9, 0.1, 10, 1, chains=2)
    dummy = ctypes.c_void_p(0x1000)
    args = lambda **o: [o.get("syn", dummy), None, o.get("n", 4), ctypes.byref(o.get("prm", prm)),
                        o.get("prob", dummy), None, None, None, o.get("chosen", dummy), None, None,
                        o.get("trace", None), o.get("ws", dummy), o.get("wsb", 0), None]
    assert lib.mcmc_decode_batch(*args(syn=None)) == -1
    assert lib.mcmc_decode_batch(*args(prob=None)) == -1
    assert lib.mcmc_decode_batch(*args(chosen=None)) == -1
    assert lib.mcmc_decode_batch(*args(ws=None, wsb=1 << 30)) == -5
    assert lib.mcmc_decode_batch(*args(wsb=16)) == -5
    assert lib.mcmc_decode_batch(*args(n=-1)) == -2
    assert lib.mcmc_decode_batch(*args(n=0)) == 0          # empty batch: nothing to do
    bad = mc.make_params(9, 0.1, 10, 1, chains=2, flags=mc.MCMC_TRACE)
    assert lib.mcmc_decode_batch(*args(prm=bad)) == -1      # trace requested, no buffer
    assert lib.mcmc_sample_errors(9, 0.1, 1, None, 0, 4, None, dummy, None, None) == -1
    assert lib.mcmc_sample_errors(9, 0.9, 1, None, 0, 4, dummy, dummy, None, None) == -2


def test_plan_rejects_invalid_items_before_allocating():
    lib = _lib._lib()
    h = ctypes.c_void_p()
    good = dict(L=9, sweeps=10, burn=0, chains=2, n_temps=1, syndrome_id=0, p=0.1,
                syn_offset=0, corr_offset=0)
    for bad, status in ((dict(L=1), -2), (dict(L=26), -2), (dict(p=0.9), -2), (dict(n_temps=3), -1),
                        (dict(chains=0), -2), (dict(sweeps=-1), -2), (dict(syn_offset=-4), -2)):
        arr = (_lib.Item * 2)()
        for i in range(2):
            for k, v in good.items():
                setattr(arr[i], k, v)
        for k, v in bad.items():
            setattr(arr[1], k, v)
        assert lib.mcmc_plan_create(arr, 2, 1, 1, ctypes.byref(h)) == status
    assert lib.mcmc_plan_create(None, 3, 1, 1, ctypes.byref(h)) == -1
    assert lib.mcmc_plan_create(None, 0, 1, 5, ctypes.byref(h)) == -1
    assert lib.mcmc_plan_destroy(None) == 0
