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
