"""The field comparison used by the GPU parity tests catches the mistakes it is
meant to catch: an FP32 copy of an oracle state passes, and a small error
confined to one PML corner, one tile-seam column, one z plane, a PEC sheet's
rim or a single node fails.  The errors are planted into a copy of the oracle's
own result, on the CPU."""
import numpy as np
import pytest

import boardgen
from _compare import FIELDS, aux_masks, compare_fields, rim_mask
from test_gpu_parity import random_state


@pytest.fixture(scope="module")
def case(oracle_mod):
    nx, ny, nz = 140, 60, 24
    eps, mask = boardgen.air(nx, ny, nz)
    eps[4:12, :, :] = 4.4
    boardgen.pec_sheet(mask, 4, 10, 50, 5, 22)
    boardgen.pec_sheet(mask, 12, 0, nx, 0, ny)
    b = boardgen.Board("cmp", nx, ny, nz, 0.5e-3, 0.5e-3, 0.2e-3, eps, mask,
                       npml=(4, 3, 2, 4, 3, 2), steps=3)
    st = random_state(oracle_mod, b, seed=11)
    ref = oracle_mod.run(b, state=st).state
    # what the library returns: FP32 values, D/B only where a PML loss keeps them
    am = aux_masks(b)
    fp32 = {}
    for n in FIELDS:
        v = ref[n].astype(np.float32).astype(np.float64)
        fp32[n] = np.where(am[n[-1]], v, 0.0) if n[0] in "db" else v
    return b, ref, fp32


def _fails(b, ref, got, check):
    with pytest.raises(AssertionError) as ei:
        compare_fields(ref, got, b, 2e-5)
    assert ei.value.args[0][1] == check, ei.value.args[0]


def _plant(fp32, ref, name, where):
    """A copy of the FP32 state whose array ``name`` carries, on the nodes
    ``where``, an error of 1.8e-5 of the array's largest value with a random sign:
    below the element-wise bound, and too small to move the whole-array norm."""
    got = dict(fp32)
    got[name] = fp32[name].copy()
    rng = np.random.default_rng(0)
    sel = got[name][where]
    sel += 1.8e-5 * np.abs(ref[name]).max() * rng.choice([-1.0, 1.0], size=sel.shape)
    got[name][where] = sel
    return got


def test_fp32_copy_passes(case):
    b, ref, fp32 = case
    rep = compare_fields(ref, fp32, b, 2e-5)
    assert set(rep) >= {"ex", "ey", "ez", "hx", "hy", "hz"}
    assert max(v[2] for v in rep.values()) < 1e-6


def test_pml_corner_error_fails(case):
    b, ref, fp32 = case
    _fails(b, ref, _plant(fp32, ref, "ex", np.s_[:3, :2, :4]), "region")   # low x/y/z corner


def test_seam_column_error_fails(case):
    b, ref, fp32 = case
    _fails(b, ref, _plant(fp32, ref, "hy", np.s_[:, 10:40, 63]), "region")    # after a 64-wide tile


def test_single_plane_error_fails(case):
    b, ref, fp32 = case
    _fails(b, ref, _plant(fp32, ref, "ez", np.s_[7, :6, :70]), "region")   # part of one plane


def test_rim_error_fails(case):
    b, ref, fp32 = case
    rim = rim_mask(b)
    assert rim.any() and not rim.all()
    # the rim layer above the island sheet at k = 4 only
    above = (np.arange(b.nz + 1) == 5)[:, None, None]
    _fails(b, ref, _plant(fp32, ref, "hz", rim & above), "region")


def test_single_node_error_fails(case):
    b, ref, fp32 = case
    got = dict(fp32)
    got["hx"] = fp32["hx"].copy()
    k, j, i = np.unravel_index(np.argmax(np.abs(ref["hx"])), ref["hx"].shape)
    got["hx"][k, j, i] += 3e-5 * np.abs(ref["hx"]).max()
    _fails(b, ref, got, "element-wise")


def test_uniform_small_error_fails_the_norm(case):
    b, ref, fp32 = case
    got = dict(fp32)
    got["ey"] = fp32["ey"] * (1.0 + 3e-5)
    _fails(b, ref, got, "whole")
