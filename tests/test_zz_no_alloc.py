"""The allocation-free probe spectrum (fdtd_probe_fft_noalloc) against
fdtd_probe_fft through the C-ABI: bitwise equal spectra on two calls in a row,
the second with a smaller transform (so the scratch keeps the first call's
larger contents), on two boards; zeros before the first step; sizes beyond the
fixed scratch are rejected with a clear error."""
import numpy as np
import pytest

import boardgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def test_noalloc_fft_equals_allocating_fft(F):
    b = boardgen.small_board(steps=3000)
    t1 = boardgen.table1_board(steps=1500, source="resistive")
    print(f"[gpu] no-alloc FFT: {b.name} {b.steps} steps, {t1.name} {t1.steps} steps", flush=True)
    g, ids = F.grid_from_board(b)
    g1, ids1 = F.grid_from_board(t1)
    try:
        z = F.fdtd_probe_fft_noalloc(g, ids[0], 4096)
        assert np.array_equal(z, np.zeros(2049, complex))       # nothing stepped yet
        F.fdtd_step_n(g, b.steps)
        F.fdtd_step_n(g1, t1.steps)
        for handle, pids, n_fft in ((g, ids, 1 << 16), (g1, ids1, 2048), (g, ids, 4096)):
            for p in pids:
                ref = F.fdtd_probe_fft(handle, p, n_fft)
                got = F.fdtd_probe_fft_noalloc(handle, p, n_fft)
                assert np.abs(ref).max() > 0
                assert np.array_equal(got, ref), (n_fft, p)
        with pytest.raises(F.FdtdError) as ei:
            F.fdtd_probe_fft_noalloc(g, ids[0], 1 << 21)
        assert ei.value.code == F.FDTD_EINVAL and "allocation-free maximum" in str(ei.value)
        with pytest.raises(F.FdtdError):
            F.fdtd_probe_fft_noalloc(g, ids[0], 2048)               # shorter than the run
    finally:
        F.fdtd_destroy_grid(g)
        F.fdtd_destroy_grid(g1)
