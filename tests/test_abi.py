"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol the header declares, and rejects bad arguments before touching a device."""
import pytest

from paper_1008_2602_amd import fdtd as F


def test_library_exports_every_header_symbol():
    syms = F.header_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(F.library(), s)]
    assert not missing, missing


def test_binding_wraps_every_header_symbol():
    for s in F.header_symbols():
        assert hasattr(F, s), s


def test_tile_shapes_listed():
    shapes = F.fdtd_tile_shapes()
    assert (64, 8, 1) in shapes and (64, 10, 2) in shapes
    assert all(tx % 64 == 0 and (tx * ty + 64 if st == 1 else 64 * ty + 128) <= 1024
               for tx, ty, st in shapes)


@pytest.mark.parametrize("kw,frag", [
    (dict(nx=1), "nx, ny, nz"),
    (dict(dx=0.0), "cell sizes"),
    (dict(courant=1.2), "courant"),
    (dict(dt=5e-12), "CFL"),
    (dict(npml=(30, 30, 8, 8, 8, 8)), "overlap"),
    (dict(npml=(-1, 8, 8, 8, 8, 8)), ">= 0"),
    (dict(max_steps=0), "max_steps"),
    (dict(pml_R=2.0), "PML parameters"),
])
def test_create_grid_rejects_bad_arguments(kw, frag):
    args = dict(nx=40, ny=40, nz=20, dx=1e-3, dy=1e-3, dz=1e-3, max_steps=10)
    args.update(kw)
    nx, ny, nz, dx, dy, dz = (args.pop(k) for k in ("nx", "ny", "nz", "dx", "dy", "dz"))
    with pytest.raises(F.FdtdError) as ei:
        F.fdtd_create_grid(nx, ny, nz, dx, dy, dz, **args)
    assert ei.value.code == F.FDTD_EINVAL
    assert frag in str(ei.value)


def test_null_handle_is_einval():
    with pytest.raises(F.FdtdError) as ei:
        F.fdtd_step_n(None, 1)
    assert ei.value.code == F.FDTD_EINVAL
    F.fdtd_destroy_grid(None)  # NULL is accepted


def test_plane_size_limit():
    """Boards past the tiled kernels' 4 GiB offset window are accepted (they step
    on the node passes from per-component bases); what is refused is a node
    plane so large that three of them (a chunk's base plane and its neighbours)
    leave 32-bit offsets.  2048 x 2048 x 600 cells pass the size checks (the call
    then fails only for want of a device here); 40000 x 40000 do not."""
    with pytest.raises(F.FdtdError) as ei:
        F.fdtd_create_grid(40000, 40000, 4, 1e-3, 1e-3, 1e-3, max_steps=1)
    assert "three node planes" in str(ei.value)
    try:
        g = F.fdtd_create_grid(2048, 2048, 600, 1e-3, 1e-3, 1e-3, max_steps=1)
    except F.FdtdError as e:
        assert "too large" not in str(e)
    else:
        F.fdtd_destroy_grid(g)
