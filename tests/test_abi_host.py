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
    assert lib.mcmc_abi_version() == 0x00010500


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


@pytest.mark.parametrize("noise,p", [(0, 0.05), (0, 0.15), (1, 0.02), (1, 0.08), (1, 0.1),
                                     (1, 0.3), (1, 0.49)])
@pytest.mark.parametrize("K,scale", [(1, 0.0), (1, 1.0), (1, 0.85), (1, 0.5), (1, 4.0),
                                     (2, 0.0), (20, 1.0)])
def test_params_tables_match_oracle(noise, p, K, scale):
    """The thresholds of a decode under each noise model equal the oracle's
    (beta* = scale * beta_bar for K = 1, the model default when scale is 0)."""
    prm = mc.make_params(9, p, 10, 1, n_temps=K, noise=noise, beta_scale=scale)
    want = tables.tables(p, K, noise, None if scale == 0.0 else scale)
    assert np.array_equal(mc.params_table(prm), want)
    if noise == 0 and scale in (0.0, 1.0):
        assert np.array_equal(mc.params_table(prm), mc.acceptance_table(p, K))


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
    (dict(flags=5), -1),
    (dict(init=3), -1), (dict(noise=2), -1), (dict(noise=1, p=0.5), -2),
    (dict(noise=1, p=0.0), -2), (dict(beta_scale=-0.5), -2), (dict(beta_scale=4.5), -2),
    (dict(beta_scale=float("nan")), -2), (dict(n_temps=2, beta_scale=0.85), -2),
])
def test_param_validation(kw, status):
    with pytest.raises(mc.McmcError) as e:
        _ws(**kw)
    assert e.value.status == status


def test_param_reserved_must_be_zero():
    prm = mc.make_params(9, 0.1, 10, 1)
    prm.reserved = 1
    with pytest.raises(mc.McmcError) as e:
        mc.workspace_size(prm, 4)
    assert e.value.status == -1
    for kw in (dict(noise=1, p=0.45), dict(n_temps=2, beta_scale=1.0), dict(beta_scale=0.85)):
        assert _ws(**kw) > 0


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
    assert lib.mcmc_sample_errors_model(9, 2, 0.1, 1, None, 0, 4, dummy, dummy, None, None) == -1
    assert lib.mcmc_sample_errors_model(9, 1, 0.6, 1, None, 0, 4, dummy, dummy, None, None) == -2
    assert lib.mcmc_sample_errors_model(9, 1, 0.1, 1, None, 0, 4, None, dummy, None, None) == -1


def test_plan_rejects_invalid_items_before_allocating():
    lib = _lib._lib()
    h = ctypes.c_void_p()
    good = dict(L=9, sweeps=10, burn=0, chains=2, n_temps=1, syndrome_id=0, p=0.1,
                syn_offset=0, corr_offset=0)
    for bad, status in ((dict(L=1), -2), (dict(L=26), -2), (dict(p=0.9), -2), (dict(n_temps=3), -1),
                        (dict(chains=0), -2), (dict(sweeps=-1), -2), (dict(syn_offset=-4), -2),
                        (dict(noise=2), -1), (dict(reserved=1), -1), (dict(noise=1, p=0.5), -2),
                        (dict(beta_scale=-0.1), -2), (dict(beta_scale=float("nan")), -2),
                        (dict(n_temps=2, beta_scale=0.85), -2)):
        arr = (_lib.Item * 2)()
        for i in range(2):
            for k, v in good.items():
                setattr(arr[i], k, v)
        for k, v in bad.items():
            setattr(arr[1], k, v)
        assert lib.mcmc_plan_create(arr, 2, 1, 1, ctypes.byref(h)) == status
    # both noise models and a lowered beta* pass validation in one plan
    arr = (_lib.Item * 2)()
    for i in range(2):
        for k, v in good.items():
            setattr(arr[i], k, v)
    arr[1].noise, arr[1].p, arr[1].beta_scale = 1, 0.45, 0.85
    assert lib.mcmc_plan_create(arr, 2, 1, 1, ctypes.byref(h)) in (0, -3, -4, -6)
    if h:
        assert lib.mcmc_plan_destroy(h) == 0
        h = ctypes.c_void_p()
    assert lib.mcmc_plan_create(None, 3, 1, 1, ctypes.byref(h)) == -1
    assert lib.mcmc_plan_create(None, 0, 1, 5, ctypes.byref(h)) == -1
    assert lib.mcmc_plan_destroy(None) == 0


@pytest.mark.parametrize("L", [2, 5, 13, 25])
def test_gate_network_sizes_match_oracle(L):
    """Parameter count and the layer layout of the C side agree with the
    oracle's parameter shapes; workspace queries are consistent."""
    from oracle import cnn
    lib = _lib._lib()
    n = ctypes.c_int64()
    assert lib.mcmc_cnn_param_count(L, ctypes.byref(n)) == 0
    assert n.value == sum(int(np.prod(s)) for _, s in cnn.param_shapes(L))
    b, bi = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.mcmc_cnn_workspace_size(L, 1000, ctypes.byref(b)) == 0
    assert lib.mcmc_cnn_infer_workspace_size(L, ctypes.byref(bi)) == 0
    offs = (ctypes.c_int64 * 7)()
    assert lib.mcmc_cnn_workspace_offsets(L, 1000, offs) == 0
    o = list(offs)
    # activations hold 1000 L^2 pixels x 32 bf16 each and do not overlap
    assert all(x % 256 == 0 for x in o) and len(set(o)) == 7
    assert o[2] - o[1] >= 1000 * L * L * 32 * 2
    assert 0 < bi.value < b.value
    assert lib.mcmc_cnn_workspace_size(L, 0, ctypes.byref(b)) == 0 and b.value == 0


def test_gate_network_rejects_before_launch():
    lib = _lib._lib()
    d = ctypes.c_void_p(0x1000)
    n = ctypes.c_int64()
    assert lib.mcmc_cnn_param_count(1, ctypes.byref(n)) == -2
    assert lib.mcmc_cnn_param_count(26, ctypes.byref(n)) == -2
    assert lib.mcmc_cnn_param_count(13, None) == -1
    big = (1 << 24) + 1
    for fn in (lib.mcmc_cnn_forward, lib.mcmc_cnn_infer):
        assert fn(13, 8, None, d, d, d, d, 1 << 30, None) == -1       # no parameters
        assert fn(13, 8, d, d, d, d, None, 0, None) == -5             # no workspace
        assert fn(13, 8, d, d, d, d, d, 16, None) == -5               # workspace too small
        assert fn(13, big, d, d, d, d, d, 1 << 30, None) == -2        # batch too large
        assert fn(1, 8, d, d, d, d, d, 1 << 30, None) == -2           # bad L
        assert fn(13, 0, None, None, None, None, None, 0, None) == 0   # empty batch
    assert lib.mcmc_cnn_backward(13, 8, d, d, d, d, ctypes.c_float(-1.0), d, None, d, 1 << 30,
                                 None) == -2                           # negative budget weight
    assert lib.mcmc_cnn_backward(13, 8, d, d, None, d, ctypes.c_float(0.5), d, None, d, 1 << 30,
                                 None) == -1                           # no class targets
    f = ctypes.c_float
    assert lib.mcmc_cnn_step(10, 0, f(1e-3), f(0.9), f(0.999), f(1e-8), d, d, d, d, None) == -2
    assert lib.mcmc_cnn_step(10, 1, f(1e-3), f(1.0), f(0.999), f(1e-8), d, d, d, d, None) == -2
    assert lib.mcmc_cnn_step(10, 1, f(1e-3), f(0.9), f(0.999), f(0.0), d, d, d, d, None) == -2
    assert lib.mcmc_cnn_step(0, 1, f(1e-3), f(0.9), f(0.999), f(1e-8), None, None, None, None,
                             None) == 0
    assert lib.mcmc_cnn_gate(8, d, f(1.5), 0, d, d, None, None) == -2
    assert lib.mcmc_cnn_gate(8, None, f(0.9), 0, d, d, None, None) == -1
    rt = lib.mcmc_gate_relative_targets
    assert rt(-1, d, d, d, None) == -2
    assert rt(0, None, None, None, None) == 0
    assert rt(4, None, d, ctypes.c_void_p(0x9000), None) == -1
    assert rt(4, d, d, ctypes.c_void_p(0x1000 + 63), None) == -1     # overlapping rows


def test_gated_config_rejected_before_allocating():
    lib = _lib._lib()
    h = ctypes.c_void_p()

    def cfg(**kw):
        c = _lib.GateConfig(L=13, n_temps=1, chains=4, burn=0, sweeps_short=13, sweeps_full=169,
                            p=0.15, seed=1, init=1, threshold=0.99, escalate=0.0, max_batch=64)
        for k, v in kw.items():
            setattr(c, k, v)
        return c
    for bad, status in ((dict(L=1), -2), (dict(p=0.8), -2), (dict(max_batch=0), -2),
                        (dict(threshold=1.5), -2), (dict(escalate=-0.1), -2),
                        (dict(escalate=2.0, chains=1), -2), (dict(class_route=2), -1),
                        (dict(class_route=1, escalate=2.0), -1),
                        (dict(sweeps_short=-1), -2), (dict(init=7), -1)):
        assert lib.mcmc_gated_create(ctypes.byref(cfg(**bad)), ctypes.byref(h)) == status, bad
    assert lib.mcmc_gated_create(None, ctypes.byref(h)) == -1
    assert lib.mcmc_gated_destroy(None) == 0


def test_gap_route_entry_points_reject_before_launch():
    lib = _lib._lib()
    d = ctypes.c_void_p(0x1000)
    sw = lib.mcmc_start_weights
    assert sw(1, 2, d, 4, d, None) == -2                 # bad L
    assert sw(13, 7, d, 4, d, None) == -1                # bad start mode
    assert sw(13, 2, d, -1, d, None) == -2
    assert sw(13, 2, None, 4, d, None) == -1
    assert sw(13, 2, None, 0, None, None) == 0           # empty batch
    fit = lib.mcmc_gate_fit_gap_table
    table = (ctypes.c_uint8 * 50)()
    p_ok = (ctypes.c_double * 2)(0.1, 0.2)
    p_bad = (ctypes.c_double * 2)(0.1, 0.8)
    assert fit(2, p_ok, d, d, 0.01, 10, None, None) == -1             # no table
    assert fit(2, None, d, d, 0.01, 10, table, None) == -1            # no rates
    assert fit(-1, p_ok, d, d, 0.01, 10, table, None) == -2
    assert fit(2, p_ok, d, d, 1.5, 10, table, None) == -2             # max_miss > 1
    assert fit(2, p_ok, d, d, 0.01, 0, table, None) == -2             # min_count < 1
    assert fit(2, p_bad, d, d, 0.01, 10, table, None) == -2           # rate out of range
    assert fit(0, None, None, None, 0.01, 10, table, None) == 0       # no samples: all NEVER
    assert list(table) == [255] * 50
    assert lib.mcmc_gated_set_gap_table(None, table) == -1


@pytest.mark.parametrize("p,pm", [(0.05, 0.05), (0.1, 0.02), (0.15, 0.3), (0.03, 0.45)])
def test_spacetime_tables_match_oracle(p, pm):
    """Space-time thresholds and xi of the C side equal the oracle's."""
    from oracle import spacetime as stm
    prm = mc.spacetime_params(5, 3, p, pm, 10, 1)
    sp, tt, always, xi = mc.spacetime_tables(prm)
    assert xi == stm.xi_of(p, pm)
    assert np.array_equal(sp, tables.acceptance_table(tables.beta_bar(p)))
    o_thr, o_always = stm.time_table(tables.beta_bar(p), stm.xi_of(p, pm))
    assert np.array_equal(always, o_always)
    assert np.array_equal(tt, np.where(o_always, 0, o_thr))


@pytest.mark.parametrize("kw,status", [
    (dict(rounds=0), -2), (dict(rounds=65), -2), (dict(p_m=0.5), -2), (dict(p_m=0.0), -2),
    (dict(p=0.8), -2), (dict(L=26), -2), (dict(chains=0), -2), (dict(sweeps=-1), -2),
    (dict(L=13, rounds=22), 0), (dict(L=25, rounds=64), 0),
])
def test_spacetime_validation(kw, status):
    base = dict(L=5, rounds=3, p=0.05, p_m=0.05, sweeps=4, seed=1, chains=2)
    base.update(kw)
    prm = mc.spacetime_params(**base)
    b = ctypes.c_size_t()
    assert _lib._lib().mcmc_spacetime_workspace_size(ctypes.byref(prm), 8, ctypes.byref(b)) == status


def test_spacetime_limits_and_reserved():
    b = ctypes.c_size_t()
    prm = mc.spacetime_params(13, 21, 0.05, 0.05, 4, 1)
    assert _lib._lib().mcmc_spacetime_workspace_size(ctypes.byref(prm), 8, ctypes.byref(b)) == 0
    prm.reserved = 3
    assert _lib._lib().mcmc_spacetime_workspace_size(ctypes.byref(prm), 8, ctypes.byref(b)) == -1
    lib = _lib._lib()
    dummy = ctypes.c_void_p(0x1000)
    assert lib.mcmc_sample_spacetime(5, 0, 0.05, 0.05, 1, 0, 4, dummy, dummy, None) == -2
    assert lib.mcmc_sample_spacetime(5, 3, 0.05, 0.05, 1, 0, 4, None, dummy, None) == -1
    good = mc.spacetime_params(5, 3, 0.05, 0.05, 4, 1)
    assert lib.mcmc_decode_spacetime(None, None, 4, ctypes.byref(good), dummy, None, None, None,
                                     None, None, dummy, None, dummy, 1 << 30, None) == -1
    assert lib.mcmc_decode_spacetime(dummy, None, 4, ctypes.byref(good), dummy, None, None, None,
                                     None, None, dummy, None, dummy, 16, None) == -5
    assert lib.mcmc_decode_spacetime(dummy, None, 0, ctypes.byref(good), dummy, None, None, None,
                                     None, None, dummy, None, None, 0, None) == 0


def test_spacetime_history_count_limit():
    """At most 2^28 histories per decode (every grid stays within 32-bit
    block counts)."""
    b = ctypes.c_size_t()
    prm = mc.spacetime_params(5, 3, 0.05, 0.05, 4, 1)
    lib = _lib._lib()
    assert lib.mcmc_spacetime_workspace_size(ctypes.byref(prm), 1 << 28, ctypes.byref(b)) == 0
    assert lib.mcmc_spacetime_workspace_size(ctypes.byref(prm), (1 << 28) + 1,
                                             ctypes.byref(b)) == -2
