"""Oracle pins of remeshing at coarse-step boundaries (Sec. 3.2.2 wavelet
criterion, Sec. 5): what the mathematics fixes about the wavelet indicator, the
refine / coarsen decisions and the intergrid transfer."""
import numpy as np
import pytest

from oracle import octree as ot
from oracle import remesh as rm
from workloads import config, mesh_spec, node_units, physical, wave_gaussian


def _poly(x, deg):
    """A tensor polynomial of degree `deg` per axis (two fields)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    u = sum((0.3 + 0.1 * k) * X ** k * Y ** (deg - k) for k in range(deg + 1)) + 0.7 * Z ** deg + 0.2
    v = (X - 0.2) ** deg * (1.0 + Y * Z) if deg >= 1 else np.ones_like(X)
    return np.stack([u, v])


def _mesh(name):
    return ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec(name)))


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_indicator_vanishes_exactly_to_degree_two(deg):
    om = _mesh("small")
    x = physical(node_units(om.anchors, om.levels, om.L), om.L)
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    f = np.stack([(X + 2 * Y - Z) ** deg + X * Y * Z ** min(deg, 2) * (deg >= 2), Y ** deg])
    w = rm.wavelet_indicator(np.moveaxis(f, 0, 1))
    if deg <= 2:
        assert w.max() < 1e-13
    else:
        assert w.max() > 1e-6


def test_parent_values_are_the_coincident_child_nodes():
    """The parent's nodes of a family are nodes of its children: a polynomial gives
    the parent's own nodal values."""
    om = _mesh("wave_c1")
    fam = rm.families(om)
    assert len(fam) > 0
    x = physical(node_units(om.anchors, om.levels, om.L), om.L)
    f = _poly(x, 4)
    for first in fam[:20]:
        par = rm.parent_values(np.moveaxis(f[:, first:first + 8], 1, 0))
        lev = int(om.levels[first]) - 1
        pa = om.anchors[first][None, :]
        xp = physical(node_units(pa, np.array([lev]), om.L), om.L)[0]
        assert np.allclose(par, _poly(xp, 4), rtol=0, atol=1e-13)


def test_transfer_identity_is_bitwise():
    om = _mesh("wave_c1")
    U = np.random.default_rng(3).standard_normal((2, om.n_oct, 5, 5, 5))
    assert np.array_equal(rm.transfer(om, om, U), U)


def _pulse_remesh(eps=1e-3):
    om = _mesh("wave_c1")
    cfg = config("wave_c1")
    U0 = wave_gaussian(om.anchors, om.levels, om.L, cfg["pulses"], sigma=cfg["sigma"])
    return om, U0, rm.remesh(om, U0, eps, 2, 4)


def test_remesh_is_balanced_tiles_and_refines_where_the_indicator_is_large():
    om, U0, new = _pulse_remesh()
    assert ot.is_balanced_bruteforce(new.anchors, new.levels, new.L)
    ot.level_grid(new.anchors, new.levels, new.L)        # tiles the domain (raises otherwise)
    leaf, fam, fw = rm.indicators(om, U0)
    # every old leaf whose indicator exceeded eps (below l_max) is covered by finer leaves now
    for i in np.nonzero((leaf > 1e-3) & (om.levels < 4))[0]:
        a, l = om.anchors[i], int(om.levels[i])
        s = 1 << (om.L - l)
        inside = ((new.anchors >= a) & (new.anchors < a + s)).all(axis=1)
        assert (new.levels[inside] > l).all()


def test_polynomials_transfer_exactly():
    """Tensor degree <= 4 data are carried exactly: degree-4 Lagrange interpolation
    into finer leaves, coincident nodes into merged parents."""
    om, U0, new = _pulse_remesh()
    assert (new.levels > 2).any() and len(new.levels) != len(om.levels)
    xo = physical(node_units(om.anchors, om.levels, om.L), om.L)
    xn = physical(node_units(new.anchors, new.levels, new.L), new.L)
    got = rm.transfer(om, new, _poly(xo, 4))
    assert np.abs(got - _poly(xn, 4)).max() < 1e-12
    # with merges: a field that is quadratic everywhere merges every family above l_min
    quad = _poly(xo, 2)
    merged = rm.remesh(om, quad, 1e-6, 2, 4)
    assert merged.n_oct < om.n_oct
    got = rm.transfer(om, merged, _poly(xo, 4))
    xm = physical(node_units(merged.anchors, merged.levels, merged.L), merged.L)
    assert np.abs(got - _poly(xm, 4)).max() < 1e-12


def test_quadratic_data_never_split():
    om = _mesh("wave_c1")
    x = physical(node_units(om.anchors, om.levels, om.L), om.L)
    new = rm.remesh(om, _poly(x, 2), 1e-9, 2, 4)
    leaf, _, _ = rm.indicators(om, _poly(x, 2))
    assert leaf.max() < 1e-9
    # no leaf got finer than the old leaf at its anchor
    kold = ot.morton_key(om.anchors[:, 0], om.anchors[:, 1], om.anchors[:, 2])
    knew = ot.morton_key(new.anchors[:, 0], new.anchors[:, 1], new.anchors[:, 2])
    o = np.searchsorted(kold, knew, side="right") - 1
    assert (new.levels <= om.levels[o]).all()
    assert (new.levels < om.levels[o]).any()        # and families merged
