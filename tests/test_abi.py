"""The C-ABI library loads and exports every entry point include/skyline.h declares.

Runs without a GPU: only calls that touch no device are made.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skyline.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sky_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_path():
    names = _declared()
    for n in ("sky_create", "sky_destroy", "sky_skyline", "sky_mlp_score", "sky_mlp_train", "sky_domcount"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2411_14968_amd as sky
    L = sky.lib()
    for n in _declared():
        assert hasattr(L, n), n


def test_opts_default_and_nparams():
    import paper_2411_14968_amd as sky
    o = sky.SkyOpts()
    sky.lib().sky_opts_default(C.byref(o))
    assert (o.partitioning, o.p, o.reps, o.n_reps, o.merge, o.presort, o.grid_filter) == (3, 16, 1, 64, 0, 2, 0)
    assert sky.lib().sky_mlp_nparams(6, 64) == 4673
    assert sky.lib().sky_mlp_nparams(8, 64) == 64 * 8 + 64 * 64 + 3 * 64 + 1


def test_create_fails_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2411_14968_amd as sky
    h = C.c_void_p()
    assert sky.lib().sky_create(C.byref(h), 0) != 0
    assert not h.value


def test_tune_defaults_and_null_context():
    import paper_2411_14968_amd as sky
    assert sky.tune_default(6) == dict(local_ppl=2, local_seg=1024, merge_ppl=2, merge_seg=1024, wg_per_cu=8)
    assert sky.tune_default(7)["local_ppl"] == 1 and sky.tune_default(7)["merge_ppl"] == 1
    t = sky.SkyTuneParams(2, 1024, 2, 1024, 8)
    L = sky.lib()
    assert L.sky_tune_set(None, 6, 1000, C.byref(t)) == -1
    assert L.sky_tune_get(None, 6, 1000, C.byref(t)) == -1
    assert L.sky_tune_load(None, b"/nonexistent") == -1
    assert L.sky_tune_save(None, b"/nonexistent") == -1
    L.sky_tune_clear(None)
