"""Host-side checks of the C-ABI library that need no GPU: every symbol the
header declares is exported, the host FE-DVR setup and tau grids agree with
the oracle, and invalid arguments are rejected before any device work."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

import paper_0911_4348_amd as negf
import workloads as W
from oracle import fedvr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(negf.LIB_PATH):
        from paper_0911_4348_amd import build
        build.build()
    return negf.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "negf_sigma2b" in names and "fedvr_build" in names and "negf_scf" in names
    assert "negf_matrix_rate" in names                  # declared in negf_measure.h
    for name in names:
        assert hasattr(L, name), name


@pytest.mark.parametrize("maker", [W.config_he, W.config_sigma_bench, W.config_h3p,
                                   lambda: W.he_1d(bounds=W.graded_bounds(100.0, 29), n_g=7)])
def test_fedvr_build_matches_oracle(L, maker):
    s = maker()
    x, Wt, T, v, V = negf.fedvr_build_system(s)
    st = fedvr.Setup(s)
    assert np.max(np.abs(x - st.x)) < 1e-13 * max(1, np.max(np.abs(st.x)))
    assert np.max(np.abs(Wt - st.W)) < 1e-13
    assert np.max(np.abs(T - st.T)) < 1e-11 * np.max(np.abs(st.T))
    assert np.max(np.abs(v - st.v)) < 1e-13
    assert np.max(np.abs(V - st.V)) < 1e-13


def test_tau_grids_match_oracle(L):
    t = negf.tau_grid("uniform", 50.0, M=1024)
    assert np.array_equal(t, fedvr.tau_uniform(50.0, 1024))
    t = negf.tau_grid("power", 100.0, u=64, p=16)
    assert np.max(np.abs(t - fedvr.tau_power(100.0, 64, 16))) < 1e-14
    assert np.all(t + t[::-1] == 100.0)


def test_sizes_and_invalid_arguments(L):
    assert negf.fedvr_size(40, 5) == 199
    with pytest.raises(negf.NegfError) as e:
        negf.fedvr_size(0, 5)
    assert e.value.code == negf.EINVAL
    with pytest.raises(negf.NegfError):
        negf.tau_grid("uniform", 1.0, M=7)
    with pytest.raises(negf.NegfError):
        negf.fedvr_build([0.0, -1.0], 4, [0.0], [1.0])
    # device entry points reject bad arguments before touching a device
    rc = L.negf_sigma2b(None, 10, 5, 2, None, None, None, 0, None)
    assert rc == negf.EINVAL
    rc = L.negf_sigma2b(C.c_void_p(1), 0, 5, 2, C.c_void_p(8), C.c_void_p(16), C.c_void_p(24), 0, None)
    assert rc == negf.EINVAL and b"n_b" in L.negf_last_error()
    rc = L.negf_sigma2b(C.c_void_p(1), 10, 5, 3, C.c_void_p(8), C.c_void_p(16), C.c_void_p(24), 0, None)
    assert rc == negf.EINVAL and b"sigma" in L.negf_last_error()
    rc = L.negf_sigma2b(C.c_void_p(1), 10, 5, 2, C.c_void_p(8), C.c_void_p(16), C.c_void_p(16), 0, None)
    assert rc == negf.EINVAL and b"alias" in L.negf_last_error()
    tau = np.array([0.0, 1.0, 1.5, 3.0])
    tg = negf.TauGrid("uniform", 3.0, tau)
    rc = L.negf_energy(C.c_void_p(1), C.byref(tg.struct), 4, 2, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                       C.c_void_p(8), 0, None, None, None)
    assert rc == negf.EINVAL and b"symmetric" in L.negf_last_error()


def test_scf_rejects_bad_options(L):
    s, keep = negf.system_struct(W.config_he())
    o = negf.OptsT(1.5, 1e-8, 10, 0, 0, 0, 1, 0.0, 0.0, 0)
    rc = L.negf_scf(C.c_void_p(1), C.byref(s), C.byref(o), None, None, None, None, None, None, 0, None, None, None)
    assert rc == negf.EINVAL and b"alpha" in L.negf_last_error()


def test_no_device_reports_enodev(L):
    try:
        import torch
        has = torch.cuda.is_available()
    except Exception:
        has = False
    if has:
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert L.negf_ctx_create(0, C.byref(h)) == negf.ENODEV


def test_batched_entry_points_reject_bad_arguments(L):
    """Host-side validation of the batched calls (no device is touched)."""
    n = (C.c_int * 2)(10, 0)
    sg = (C.c_int * 2)(2, 2)
    ptrs = (C.c_void_p * 2)(8, 16)
    outs = (C.c_void_p * 2)(24, 32)
    rc = L.negf_sigma2b_batched(C.c_void_p(1), 2, n, 5, sg, ptrs, ptrs, outs, 0, None)
    assert rc == negf.EINVAL and b"n_b[1]" in L.negf_last_error()
    n[1] = 10
    rc = L.negf_sigma2b_batched(C.c_void_p(1), 2, n, 5, sg, ptrs, ptrs, ptrs, 0, None)
    assert rc == negf.EINVAL and b"alias" in L.negf_last_error()
    rc = L.negf_sigma2b_batched(C.c_void_p(1), 0, n, 5, sg, ptrs, ptrs, outs, 0, None)
    assert rc == negf.EINVAL
    rc = L.negf_sigma2b_batched_set_config(C.c_void_p(1), 2, n, 0, 11)
    assert rc == negf.EINVAL
    rc = L.negf_hf_batched(C.c_void_p(1), 0, 10, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 2.0, 2, 10.0, 1e-10,
                           10, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None, None, None, None)
    assert rc == negf.EINVAL


def test_scf_batched_requires_one_tau_grid(L):
    a, ka = negf.system_struct(W.config_he())
    b, kb = negf.system_struct(W.config_he().with_(M=64))
    arr = (negf.SystemT * 2)(a, b)
    o = negf.OptsT(0.3, 1e-8, 10, 0, 0, 0, 1, 0.0, 0.0, 0)
    rc = L.negf_scf_batched(C.c_void_p(1), 2, arr, C.byref(o), None, None, None, None, None, None, None, 0, None,
                            None, None, None)
    assert rc == negf.EINVAL and b"same tau grid" in L.negf_last_error()


def test_matrix_rate_rejects_bad_arguments(L):
    """negf_matrix_rate validates on the host before touching a device."""
    tf, ghz = C.c_double(), C.c_double()
    rc = L.negf_matrix_rate(None, 0, C.byref(tf), C.byref(ghz), None)
    assert rc == negf.EINVAL and b"ctx" in L.negf_last_error()
    rc = L.negf_matrix_rate(C.c_void_p(1), 7, C.byref(tf), C.byref(ghz), None)
    assert rc == negf.EINVAL and b"dtype" in L.negf_last_error()
    rc = L.negf_matrix_rate(C.c_void_p(1), 0, None, C.byref(ghz), None)
    assert rc == negf.EINVAL


def test_issue_probe_rejects_bad_arguments(L):
    """negf_f64_issue_probe validates on the host before touching a device."""
    ms, tm, tv = C.c_double(), C.c_double(), C.c_double()
    rc = L.negf_f64_issue_probe(None, 8, 0, C.byref(ms), C.byref(tm), C.byref(tv), None)
    assert rc == negf.EINVAL and b"ctx" in L.negf_last_error()
    rc = L.negf_f64_issue_probe(C.c_void_p(1), 0, 0, C.byref(ms), C.byref(tm), C.byref(tv), None)
    assert rc == negf.EINVAL and b"chain counts" in L.negf_last_error()
    rc = L.negf_f64_issue_probe(C.c_void_p(1), 8, 0, None, C.byref(tm), C.byref(tv), None)
    assert rc == negf.EINVAL


def test_bf16_slice_limit_checked_on_host(L):
    """NEGF_BF16 takes at most 65535 slices; the limit is checked before any device work."""
    fake = C.c_void_p(1)
    rc = L.negf_sigma2b(fake, 10, 70000, 2, C.c_void_p(8), C.c_void_p(16), C.c_void_p(24), negf.BF16, None)
    assert rc == negf.EINVAL and b"65535" in L.negf_last_error()
    n = (C.c_int * 1)(10)
    sg = (C.c_int * 1)(2)
    ptrs = (C.c_void_p * 1)(8)
    outs = (C.c_void_p * 1)(24)
    Gs = (C.c_void_p * 1)(16)
    rc = L.negf_sigma2b_batched(fake, 1, n, 70000, sg, ptrs, Gs, outs, negf.BF16, None)
    assert rc == negf.EINVAL and b"65535" in L.negf_last_error()


def test_harmonic_trap_setup_matches_oracle(L):
    s = W.harmonic_trap(n_elec=20.0, omega=0.8, half_width=10.0, n_e=21, n_g=5)
    x, Wt, T, v, V = negf.fedvr_build_system(s)
    st = fedvr.Setup(s)
    assert np.max(np.abs(v - st.v)) < 1e-13 * np.max(np.abs(st.v))
    assert np.max(np.abs(V - st.V)) < 1e-13
    with pytest.raises(negf.NegfError):
        negf.fedvr_build(s.bounds, s.n_g, [], [], omega=-1.0)


def test_density_at_matches_oracle(L):
    from oracle import observables as O, hf as H
    s = W.config_he()
    st = fedvr.Setup(s)
    r = H.hartree_fock(st.h, st.V, 2.0, 2, s.beta)
    xs = np.concatenate([np.linspace(-10.5, 10.5, 57), st.x, st.grid.bounds])
    got = negf.density_at(s.bounds, s.n_g, r.rho, 2, xs)
    inside = (xs >= s.bounds[0]) & (xs <= s.bounds[-1])
    ref = O.density_at(st.grid, r.rho, 2, xs[inside])
    assert np.max(np.abs(got[inside] - ref)) < 1e-12 * np.max(ref)
    assert np.all(got[~inside] == 0.0)
    with pytest.raises(negf.NegfError):
        negf.density_at(s.bounds, s.n_g, r.rho, 3, xs)


def test_noalloc_rejects_on_the_host(L):
    """The allocation-free Sigma-2B entry checks its limits before touching a device."""
    p = C.c_void_p(8)
    rc = L.negf_sigma2b_noalloc(C.c_void_p(1), 8, 65537, 2, p, C.c_void_p(16), C.c_void_p(24), negf.F32, None)
    assert rc == negf.EINVAL and b"allocation-free" in L.negf_last_error()
    rc = L.negf_sigma2b_noalloc(C.c_void_p(1), 8, 5, 2, p, C.c_void_p(16), C.c_void_p(24), negf.BF16, None)
    assert rc == negf.EINVAL and b"bf16" in L.negf_last_error()
