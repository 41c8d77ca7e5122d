"""Refinement layouts of the AMR experiments of Section 3 (CPU).

The band layouts (ILR and VLR, D2 and D2,2) are pinned to the zone and leaf
counts printed in Tables 8 and 9: within 1% at N_k = 128, where the lattice
is coarse against the band, and within 0.25% from N_k = 256 on.
"""
import os

import numpy as np
import pytest

import diskgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows():
    out = []
    for l in open(os.path.join(GOLDEN, "tables8_9_zones.txt")):
        if l.strip() and not l.startswith("#"):
            k, d, lv, n, z, e = l.split()
            out.append((k, d, int(lv), int(n), int(z), int(e)))
    return out


@pytest.mark.parametrize("kind", ["ilr", "vlr"])
@pytest.mark.parametrize("disk", ["d2", "d22"])
@pytest.mark.parametrize("levels", [2, 3])
def test_zone_and_leaf_counts_match_tables_8_9(kind, disk, levels):
    gen = diskgen.ilr_layout if kind == "ilr" else diskgen.vlr_layout
    for k, d, lv, n, zones, leaves in _rows():
        if (k, d, lv) != (kind, disk, levels) or n > 512:
            continue
        lay = gen(n, levels, disk)
        tol = 0.01 if n == 128 else 0.0025
        assert abs(lay.total() / zones - 1) < tol, (n, lay.total(), zones)
        assert abs(lay.nleaves() / leaves - 1) < tol, (n, lay.nleaves(), leaves)


def test_zone_counts_large_base():
    # the 2048 base of Table 8 (ILR, D2, 3 levels): 6 171 680 zones
    lay = diskgen.ilr_layout(2048, 3, "d2")
    assert abs(lay.total() / 6171680 - 1) < 0.001


@pytest.mark.parametrize("gen", [diskgen.ilr_layout, diskgen.vlr_layout])
def test_band_layouts_nest_and_tile(gen):
    lay = gen(128, 3, "d22")
    assert lay.validate()
    leaf = lay.leaf_mask()
    assert abs(lay.areas()[leaf].sum() - 4.0) < 1e-12
    # refined cells lie in the band: every level-1 patch cell centre is within
    # the base band of a disk edge (plus half a base cell)
    h0 = 2.0 / 128
    for b in lay.blocks()[1:]:
        if b.level != 1:
            continue
        xs = b.x0 + (np.arange(b.nx) + 0.5) * b.h
        ys = b.y0 + (np.arange(b.ny) + 0.5) * b.h
        XX, YY = np.meshgrid(xs, ys)
        d = np.minimum(np.abs(np.hypot(XX, YY - 0.5) - 0.25), np.abs(np.hypot(XX, YY + 0.5) - 0.25))
        band = 0.8 * (0.05 if gen is diskgen.ilr_layout else 0.2)
        assert d.max() < band + 0.75 * h0


def test_band_layout_patches_are_row_runs():
    # one row of refined base cells -> patches of 2 x 2k children, disjoint
    lay = diskgen.band_layout(64, 2, [(0.0, 0.0)], 0.5, [0.04])
    assert all(p.ny == 2 and p.level == 1 for p in lay.patches)
    assert lay.validate()


def test_request_pool_layouts_are_valid_and_in_range():
    """The served-stream workload: every layout is properly nested, its
    finest lattice fits the 8192-point transform limit, and its patch count
    lies in 4..256 when refined."""
    for lay, prof in diskgen.request_pool(0, count=16):
        assert lay.validate()
        assert lay.n0 in (128, 256, 512, 1024, 2048)
        assert lay.n_finest <= 4096
        if lay.nlevels > 1:
            assert 1 <= len(lay.patches) <= 256
        s, dx, dy = lay.sample(prof)
        assert np.all(np.isfinite(s)) and np.all(s >= 0)
        assert s.size == lay.total()


def test_batch_disks_shapes_and_seeding():
    a = diskgen.batch_disks(0)
    b = diskgen.batch_disks(0)
    assert len(a) == 64
    for (n, s, dx, dy), (n2, s2, _, _) in zip(a, b):
        assert n in (64, 128, 256, 512, 1024) and n == n2
        assert s.shape == (n, n) and dx.shape == (n, n) and dy.shape == (n, n)
        assert np.array_equal(s, s2)
