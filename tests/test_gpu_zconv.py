"""The z-convergence study of the Results section on the HIP path: the whole
family (1 to 15 cells across the dielectric) advanced together by one batched
call, against the FP64 oracle (probe relative L2 <= 1e-4), and the convergence
it shows equal to the oracle's."""
import numpy as np
import pytest

import boardgen
from _util import rel_l2
from test_gpu_parity import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def _metrics(series, ref):
    rel = [np.linalg.norm(series[p] - ref[p]) / np.linalg.norm(ref[p]) for p in range(len(ref))]
    peak = [abs(np.abs(series[p]).max() - np.abs(ref[p]).max()) / np.abs(ref[p]).max()
            for p in range(len(ref))]
    return np.array(rel), np.array(peak)


def test_z_convergence_family_batched(F, oracle_mod):
    steps = 4000
    boards = [boardgen.zconv_board(n, steps=steps) for n in range(1, 16)]
    announce(f"z-convergence family: {len(boards)} boards, {steps} steps, one batched call")
    hs = [F.grid_from_board(b, max_steps=steps) for b in boards]
    try:
        F.fdtd_step_many([g for g, _ in hs], [steps] * len(hs))
        F.fdtd_synchronize(hs[0][0])
        gpu = {b.meta["n_diel"]: np.stack([F.fdtd_get_probe(g, p, steps) for p in ids]).astype(np.float64)
               for b, (g, ids) in zip(boards, hs)}
    finally:
        for g, _ in hs:
            F.fdtd_destroy_grid(g)
    ref = {}
    for n in (1, 2, 15):
        announce(f"z-convergence oracle n={n}")
        ref[n] = oracle_mod.run(boards[n - 1], threads=16).probes
        for p in range(3):
            assert rel_l2(gpu[n][p], ref[n][p]) <= 1e-4, (n, p)
    # the convergence the GPU shows is the oracle's
    for n in (1, 2):
        g_rel, g_peak = _metrics(gpu[n], gpu[15])
        o_rel, o_peak = _metrics(ref[n], ref[15])
        assert np.abs(g_rel - o_rel).max() < 2e-4 and np.abs(g_peak - o_peak).max() < 2e-4
    rel = np.array([_metrics(gpu[n], gpu[15])[0] for n in range(1, 15)])
    assert np.all(np.diff(rel[:, 2]) < 0)           # far corner: monotone in n
    assert rel[1].max() < 5e-3 and _metrics(gpu[2], gpu[15])[1][2] < 1e-3
