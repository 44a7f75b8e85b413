"""CPU checks of the C ABI: the library loads, exports every function that
include/lsd.h declares, and rejects invalid configurations on the host
(no device work is started by any call here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lsd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_02455_amd import lsd
    return lsd.load()


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("lsd_init_system", "lsd_draft_steps", "lsd_verify_window", "lsd_accept_rollback"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2606_02455_amd import lsd
    assert set(_declared()) == set(lsd.EXPORTS)


def _cfg(lsd, w, **over):
    cfg = lsd.Config()
    keep = dict(off=np.ascontiguousarray(w.atom_offsets, np.int32),
                box=np.ascontiguousarray(w.box, np.float64),
                mass=np.ascontiguousarray(w.species_mass, np.float64))
    cfg.n_atoms, cfg.n_replicas = w.n_atoms, w.n_replicas
    cfg.atom_offsets = keep["off"].ctypes.data_as(C.POINTER(C.c_int32))
    cfg.box = keep["box"].ctypes.data_as(C.POINTER(C.c_double))
    cfg.species_mass = keep["mass"].ctypes.data_as(C.POINTER(C.c_double))
    cfg.n_species = 1
    cfg.dt, cfg.gamma, cfg.kT, cfg.force_unit, cfg.skin = w.dt, w.gamma, w.kT, 1.0, 0.3
    cfg.k_max, cfg.mode, cfg.seed = w.K, 0, 1
    cfg.target.kind, cfg.target.cutoff, cfg.target.epsilon, cfg.target.sigma = 1, 2.5, 1.0, 1.0
    cfg.draft.kind, cfg.draft.cutoff, cfg.draft.epsilon, cfg.draft.sigma = 1, 1.5, 1.0, 1.0
    for k, v in over.items():
        setattr(cfg, k, v)
    return cfg, keep


def test_workspace_size_and_validation(lib):
    from paper_2606_02455_amd import lsd
    from paper_2606_02455_amd import workloads as W
    w = W.config("c2")
    cfg, keep = _cfg(lsd, w)
    n = C.c_size_t()
    assert lib.lsd_workspace_size(C.byref(cfg), C.byref(n)) == 0
    # window + lists dominate: at least K frames of 16 + 12*3 bytes per atom
    assert n.value > w.K * w.n_atoms * 52
    for field, bad in (("gamma", 0.0), ("kT", -1.0), ("dt", 0.0), ("skin", 0.0), ("k_max", 65),
                       ("k_max", 0), ("mode", 7)):
        c2, _ = _cfg(lsd, w, **{field: bad})
        assert lib.lsd_workspace_size(C.byref(c2), C.byref(n)) == -1
        assert lib.lsd_last_error().decode() != ""


def test_box_must_be_binary32_and_larger_than_list_radius(lib):
    from paper_2606_02455_amd import lsd
    from paper_2606_02455_amd import workloads as W
    w = W.config("c1")
    box = np.array([4.3088693618774414 + 1e-12])  # not a binary32 value
    cfg, keep = _cfg(lsd, w)
    cfg.box = box.ctypes.data_as(C.POINTER(C.c_double))
    n = C.c_size_t()
    assert lib.lsd_workspace_size(C.byref(cfg), C.byref(n)) == -1
    small = np.array([2.5])
    cfg.box = small.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.lsd_workspace_size(C.byref(cfg), C.byref(n)) == -1
    assert "exceed" in lib.lsd_last_error().decode()


def test_init_rejects_null_buffers(lib):
    from paper_2606_02455_amd import lsd
    from paper_2606_02455_amd import workloads as W
    w = W.config("c1")
    cfg, keep = _cfg(lsd, w)
    buf = lsd.Buffers()
    h = C.c_void_p()
    assert lib.lsd_init_system(C.byref(cfg), C.byref(buf), None, C.byref(h)) == -1
    assert not h.value


def test_calls_on_null_handle_fail_cleanly(lib):
    assert lib.lsd_draft_steps(None, 4, None) == -1
    assert lib.lsd_verify_window(None, None) == -1
    assert lib.lsd_accept_rollback(None, None, None) == -1
    assert lib.lsd_destroy(None) == 0


def test_fit_pair_solve_matches_least_squares(lib):
    # host-only: Cholesky solve of extended normal equations [A|y]^T [A|y]
    from paper_2606_02455_amd import lsd
    rng = np.random.default_rng(3)
    A = rng.normal(size=(200, 12))
    y = rng.normal(size=200)
    Ae = np.concatenate([A, y[:, None]], axis=1)
    G = Ae.T @ Ae
    w = lsd.fit_pair_solve(G, ridge=0.0)
    ref, *_ = np.linalg.lstsq(A, y, rcond=None)
    assert np.allclose(w, ref, rtol=1e-10, atol=1e-12)
    # ridge: (A^T A + lam I) w = A^T y with lam = ridge * trace / P
    lam = 0.1 * np.trace(A.T @ A) / 12
    wr = lsd.fit_pair_solve(G, ridge=0.1)
    assert np.allclose(wr, np.linalg.solve(A.T @ A + lam * np.eye(12), A.T @ y), rtol=1e-10)
    # an unobserved column makes the system singular without a ridge
    A[:, 3] = 0.0
    Ae = np.concatenate([A, y[:, None]], axis=1)
    with pytest.raises(lsd.LSDError):
        lsd.fit_pair_solve(Ae.T @ Ae, ridge=0.0)
    assert np.isfinite(lsd.fit_pair_solve(Ae.T @ Ae, ridge=1e-8)).all()


def test_net_parameter_layout(lib, ora):
    # host-only: the parameter count agrees with the oracle's layout, sizes
    # outside the supported range give 0, and the initial parameters are the
    # pair draft (W2 = 0, c = pair weights)
    from oracle.net import NetDraft
    from paper_2606_02455_amd import lsd
    for S, B in ((1, 1), (3, 8), (3, 16), (4, 16)):
        assert lsd.net_param_count(S, B) == NetDraft.count(S, B)
    for S, B in ((0, 8), (5, 4), (1, 17), (2, 0)):
        assert lsd.net_param_count(S, B) == 0
    pw = np.arange(6 * 8, dtype=np.float64)
    p = lsd.net_init_params(3, 8, pair_weights=pw, seed=2)
    W1, b1, W2, c = NetDraft(3, 8, 4.0, p.astype(np.float64)).split()
    assert np.all(W2 == 0) and np.all(b1 == 0) and np.array_equal(c.ravel(), pw)
    assert np.std(W1) > 0.1


def test_learned_draft_configuration_is_validated(lib):
    # host-only: the workspace query validates the draft like init does
    from paper_2606_02455_amd import lsd
    from paper_2606_02455_amd import workloads as W
    w = W.triatomic_liquid(64, seed=3)
    weights = np.zeros(lsd.net_param_count(3, 16), np.float32)

    def cfg_with(**net):
        cfg, keep = _cfg(lsd, w, n_species=3)
        d = cfg.draft
        d.kind, d.cutoff, d.weights = lsd.POT_NET, 4.0, weights.ctypes.data
        d.n_model_species, d.n_basis, d.precision = 3, 16, lsd.PREC_BF16
        for k, v in net.items():
            setattr(d, k, v)
        return cfg, keep

    n = C.c_size_t()
    cfg, keep = cfg_with()
    assert lib.lsd_workspace_size(C.byref(cfg), C.byref(n)) == 0, lib.lsd_last_error()
    bad = [dict(n_basis=17), dict(n_basis=0), dict(n_model_species=5),
           dict(n_model_species=2),   # fewer than the system's species
           dict(precision=3), dict(precision=lsd.PREC_FP8),   # FP8 without calibration
           dict(cutoff=0.0), dict(weights=None)]
    for b in bad:
        cfg, keep = cfg_with(**b)
        assert lib.lsd_workspace_size(C.byref(cfg), C.byref(n)) == -1, b
        assert lib.lsd_last_error().decode() != ""
    cfg, keep = cfg_with(precision=lsd.PREC_FP8)
    cfg.draft.act_amax[0], cfg.draft.act_amax[1] = 2.0, 1.5
    assert lib.lsd_workspace_size(C.byref(cfg), C.byref(n)) == 0, lib.lsd_last_error()
    # drafts are never targets
    cfg, keep = cfg_with()
    cfg.target = cfg.draft
    assert lib.lsd_workspace_size(C.byref(cfg), C.byref(n)) == -5


def test_autotune_and_net_calls_on_null_handle_fail_cleanly(lib):
    ch = C.c_int32()
    assert lib.lsd_autotune_verify(None, 8, 1, C.byref(ch), None, None) == -1
    assert lib.lsd_set_verify_variant(None, 8, 2) == -1
    assert lib.lsd_net_train_accumulate(None, None, 0, 0, None, 0, None, None) == -1
    assert lib.lsd_net_adam_step(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None) == -1
    assert lib.lsd_pipeline_submit(None, None) == -1
