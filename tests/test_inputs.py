"""Host-side input generators: the closed-pore filter of the sphere-pack masks."""
import numpy as np

from paper_1804_07588_amd import workloads as W


def test_closed_single_node_cavity_is_filled():
    m = np.zeros((9, 9, 12), dtype=np.uint8)
    m[2:7, 2:7, 4:9] = 1
    m[4, 4, 6] = 0  # one gas node walled in on all 18 link directions
    f = W.fill_closed_pores(m, periodic=(0, 1, 1))
    assert f[4, 4, 6] == 1
    assert int(f.sum()) == int(m.sum()) + 1


def test_edge_link_keeps_a_node_open():
    # a node joined to the open gas through an edge diagonal only stays gas:
    # D3Q19 streams along (1, 1, 0)
    m = np.ones((5, 6, 8), dtype=np.uint8)
    m[:, :, 0:2] = 0
    m[2, 3, 2] = 0          # face-adjacent to the open region
    m[2, 4, 3] = 0          # edge-adjacent to (2, 3, 2) only
    m[2, 2, 4] = 0          # its only gas neighbours would need a two-node jump
    f = W.fill_closed_pores(m, periodic=(0, 1, 1))
    assert f[2, 3, 2] == 0 and f[2, 4, 3] == 0
    assert f[2, 2, 4] == 1


def test_periodic_faces_join_pores():
    m = np.ones((5, 8, 10), dtype=np.uint8)
    m[:, :, 0] = 0
    m[2, 7, 1:5] = 0        # channel from the inlet plane along y = ny-1
    m[2, 0, 4:7] = 0        # continues across the periodic y face
    f = W.fill_closed_pores(m, periodic=(0, 1, 1))
    assert np.all(f[2, 0, 4:7] == 0)
    g = W.fill_closed_pores(m, periodic=(0, 0, 1))
    assert np.all(g[2, 0, 4:7] == 1)  # without the y wrap the piece is closed


def test_bed_mask_only_loses_closed_cavities():
    raw, n_raw = W.sphere_pack_mask(48, radius=6.0, porosity=0.6, seed=7, buffer=4,
                                    fill_closed=False)
    m, n = W.sphere_pack_mask(48, radius=6.0, porosity=0.6, seed=7, buffer=4)
    assert n == n_raw
    assert np.all(m >= raw)
    # every node that was filled was gas with no solid-free link path to x = 0
    changed = np.argwhere(m != raw)
    for z, y, x in changed:
        assert raw[z, y, x] == 0
    # the open gas still spans inlet to outlet
    assert np.any(m[:, :, 0] == 0) and np.any(m[:, :, -1] == 0)
    assert W.fill_closed_pores(m, periodic=(0, 1, 1)).sum() == m.sum()
