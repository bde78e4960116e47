"""The C-ABI library without a GPU: it loads, exports every symbol that
include/kfvm.h declares, rejects bad arguments before touching the device, and
its binary128 weight builder agrees with the oracle's 50-digit tables."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2401_16543_amd import kfvm
    return kfvm.load_library()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "kfvm.h")).read()
    declared = set(re.findall(r"\b(kfvm_\w+)\s*\(", hdr))
    assert len(declared) >= 15
    for name in sorted(declared):
        assert hasattr(lib, name), name


def test_binding_names_follow_the_header():
    from paper_2401_16543_amd import kfvm
    hdr = open(os.path.join(ROOT, "include", "kfvm.h")).read()
    declared = set(re.findall(r"\b(kfvm_\w+)\s*\(", hdr))
    assert declared == set(kfvm.EXPORTED)


@pytest.mark.parametrize("d,R", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_weight_builder_matches_oracle(lib, d, R):
    from oracle import weights as W
    from paper_2401_16543_amd import kfvm
    got = kfvm.weights_build(d, R)
    T = W.tables(d, R)
    off = 0
    for tab in T["weights"]:
        blk = got[off:off + tab.size].reshape(tab.shape)
        off += tab.size
        scale = np.abs(tab).max(axis=1, keepdims=True)
        # within 2 ulp of each row's largest entry; rows that vanish by symmetry stay ~0
        assert np.all(np.abs(blk - tab) <= 2 * np.finfo(float).eps * scale + 1e-30)
    assert off == got.size


def test_init_rejects_bad_arguments_without_a_device(lib):
    from paper_2401_16543_amd import kfvm
    h = C.c_void_p()
    mesh = kfvm._Mesh()
    mesh.dim = 4
    assert lib.kfvm_init(C.byref(h), C.byref(mesh), 5, 1.4, None) == kfvm.KFVM_ERR_ARG
    mesh.dim = 2
    mesh.n[:] = [64, 64, 1]
    mesh.dx[:] = [1 / 64, 1 / 64, 1.0]
    assert lib.kfvm_init(C.byref(h), C.byref(mesh), 6, 1.4, None) == kfvm.KFVM_ERR_ARG
    assert lib.kfvm_init(C.byref(h), C.byref(mesh), 5, 0.9, None) == kfvm.KFVM_ERR_ARG
    mesh.n[:] = [5, 64, 1]
    assert lib.kfvm_init(C.byref(h), C.byref(mesh), 5, 1.4, None) == kfvm.KFVM_ERR_ARG
    assert b"2R + 2" in lib.kfvm_last_error(None)


def test_init_rejects_foreign_weight_layout(lib):
    from oracle import weights as W
    from paper_2401_16543_amd import kfvm
    T = dict(W.tables(2, 2))
    T["members"] = [m[::-1].copy() for m in T["members"]]      # same sizes, wrong order
    wp, keep = kfvm.KFVM._pack_weights(T)
    h = C.c_void_p()
    mesh = kfvm._Mesh()
    mesh.dim = 2
    mesh.n[:] = [32, 32, 1]
    mesh.dx[:] = [1 / 32, 1 / 32, 1.0]
    assert lib.kfvm_init(C.byref(h), C.byref(mesh), 5, 1.4, wp) == kfvm.KFVM_ERR_ARG
    assert b"layout" in lib.kfvm_last_error(None)


def test_length_scale_init_rejects_bad_values_without_a_device(lib):
    from paper_2401_16543_amd import kfvm
    h = C.c_void_p()
    mesh = kfvm._Mesh()
    mesh.dim = 2
    mesh.n[:] = [64, 64, 1]
    mesh.dx[:] = [1 / 64, 1 / 64, 1.0]
    for ell in (0.0, -1.0, float("nan"), float("inf"), 101.0):
        assert lib.kfvm_init_length_scale(C.byref(h), C.byref(mesh), 5, 1.4, ell) == kfvm.KFVM_ERR_ARG
        assert not h.value
    assert b"ell_hat" in lib.kfvm_last_error(None)


def _unit_cell_average(c, a):
    # average of x^a over the unit cell [c - 1/2, c + 1/2]
    return ((c + 0.5) ** (a + 1) - (c - 0.5) ** (a + 1)) / (a + 1)


@pytest.mark.parametrize("d,R", [(2, 2), (2, 3), (3, 2), (3, 3)])
@pytest.mark.parametrize("ell", [2.0, 20.0])
def test_tables_at_other_length_scales_keep_polynomial_exactness(lib, d, R, ell):
    """At any kernel length scale the full-stencil rows reproduce every
    polynomial of degree 2R - 1 at the face points (section 2.1: the monomial
    part fixes the order independently of l), checked on exact cell averages
    of the monomials; the error bound scales with the rows' largest weight."""
    import itertools
    from oracle import weights as W
    from paper_2401_16543_amd import kfvm
    T = W.tables(d, R)
    s0 = np.asarray(T["s0"], dtype=float)
    pts = np.array([[float(v) for v in p] for p in W.face_points(d, R)])
    deg = 2 * R - 1
    mons = [m for m in itertools.product(range(deg + 1), repeat=d) if sum(m) <= deg]
    A = np.array([[np.prod([_unit_cell_average(s0[h, i], m[i]) for i in range(d)]) for m in mons]
                  for h in range(len(s0))])
    V = np.array([[np.prod([pts[j, i] ** m[i] for i in range(d)]) for m in mons] for j in range(len(pts))])
    flat = kfvm.weights_build(d, R, ell)
    r = flat[:T["weights"][0].size].reshape(T["weights"][0].shape)[:len(pts)]
    assert np.abs(r @ A - V).max() <= 1e-13 * max(1.0, np.abs(r).max())
    assert np.abs(r - kfvm.weights_build(d, R, 5.0)[:r.size].reshape(r.shape)).max() > 1e-6   # l does change them


def test_weight_builder_matches_oracle_at_another_length_scale(lib):
    """The library's binary128 tables at l = 20 cells against the oracle's
    50-digit solve at the same l, within 2 ulp of each row's largest entry."""
    from oracle import weights as W
    from paper_2401_16543_amd import kfvm
    d, R = 2, 2
    got = kfvm.weights_build(d, R, 20.0)
    off = 0
    for q in range(len(W.tables(d, R)["weights"])):
        tab = W.stencil_weights(d, R, q, ell_hat=20)
        blk = got[off:off + tab.size].reshape(tab.shape)
        off += tab.size
        scale = np.abs(tab).max(axis=1, keepdims=True)
        assert np.all(np.abs(blk - tab) <= 2 * np.finfo(float).eps * scale + 1e-30)
    assert off == got.size
