"""The C-ABI library loads without a GPU and exports every entry point that
include/*.h declares; argument validation that needs no device work."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(pk_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    d = declared()
    for n in ["pk_create", "pk_destroy", "pk_last_error", "pk_robot_upload", "pk_fk",
              "pk_residual_jacobian", "pk_ik_solve"]:
        assert n in d


def test_library_exports_every_declared_symbol():
    import paper_2505_03728_amd as pk
    L = pk.lib()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(pk.exported_symbols()) <= set(declared())


def test_null_context_errors_without_gpu():
    import paper_2505_03728_amd as pk
    L = pk.lib()
    assert L.pk_robot_upload(None, None, None) == -1
    assert b"ctx is NULL" in L.pk_last_error(None)
    assert L.pk_destroy(None) == 0
    assert L.pk_ik_beam(None, 0, 1, None, None, None, None, None, None, None) == -1
    assert b"pk_ik_beam: ctx is NULL" in L.pk_last_error(None)


def test_pack_targets_layout():
    import numpy as np
    import paper_2505_03728_amd as pk
    tg = np.arange(2 * 3 * 7, dtype=np.float64).reshape(2, 3, 7)
    P = pk.pack_targets([0, 1, 0], tg)
    assert P.shape == (7 + 3 + 7, 2)
    np.testing.assert_array_equal(P[:7, 1], tg[1, 0])
    np.testing.assert_array_equal(P[7:10, 0], tg[0, 1, :3])
    np.testing.assert_array_equal(P[10:, 1], tg[1, 2])
