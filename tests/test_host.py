"""Host-side logic of the library that needs no GPU: domain construction
(fluid list, node order, coordinates), argument validation and call-order
errors of the C ABI."""

import numpy as np
import pytest

import synth


def _lbm():
    from paper_2101_11107_amd import lbm
    lbm.load()
    return lbm


def test_fluid_list_and_tile_order():
    lbm = _lbm()
    case = synth.pipe_case()
    dom = lbm.lbm_create_domain(case.mask, case.periodic, lbm.LBM_F64, 0)
    try:
        assert lbm.lbm_fluid_count(dom) == 20224
        xyz = lbm.lbm_fluid_coords(dom)
        # exactly the fluid cells, each once
        got = np.zeros_like(case.mask)
        got[xyz[:, 2], xyz[:, 1], xyz[:, 0]] += 1
        assert np.array_equal(got, (case.mask == synth.FLUID).astype(got.dtype))
        # rows grouped in 8 x 8 tiles of the (y, z) plane, x increasing inside a row
        key = [((z // 8) * 100 + (y // 8), z % 8, y % 8, x) for x, y, z in xyz]
        assert key == sorted(key)
        assert lbm.lbm_device_bytes(dom) > 2 * 27 * 8 * 20224
    finally:
        lbm.lbm_destroy(dom)


@pytest.mark.parametrize("tile", [1, 4, 8, 16, 32])
def test_row_tile_option_changes_only_the_order(tile):
    """lbm_create_domain_ex takes the (y, z) rows in tiles of the given edge:
    the same fluid cells in another order (edge 8 is the default order), with
    or without curved-wall links."""
    lbm = _lbm()
    case = synth.random_tiny_case(4, nx=20, ny=37, nz=21)
    ref = lbm.lbm_create_domain(case.mask, case.periodic, lbm.LBM_F32, 0)
    links = synth.wall_links(case.mask, case.periodic)
    doms = [lbm.lbm_create_domain_ex(case.mask, case.periodic, lbm.LBM_F32, None, None, tile, 0),
            lbm.lbm_create_domain_ex(case.mask, case.periodic, lbm.LBM_F32, links, np.full(len(links), 0.3),
                                     tile, 0)]
    try:
        want = lbm.lbm_fluid_coords(ref)
        for dom in doms:
            xyz = lbm.lbm_fluid_coords(dom)
            assert sorted(map(tuple, xyz)) == sorted(map(tuple, want))
            key = [((z // tile) * 100 + (y // tile), z % tile, y % tile, x) for x, y, z in xyz]
            assert key == sorted(key)
            if tile == 8:
                assert np.array_equal(xyz, want)
    finally:
        for d in (ref, *doms):
            lbm.lbm_destroy(d)


@pytest.mark.parametrize("tile", [0, 3, 64, -8])
def test_row_tile_option_rejects_other_edges(tile):
    lbm = _lbm()
    case = synth.random_tiny_case(1)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create_domain_ex(case.mask, case.periodic, lbm.LBM_F32, None, None, tile, 0)
    assert e.value.code == lbm.LBM_EINVAL


def test_aneurysm_fluid_counts():
    lbm = _lbm()
    for n, expect in ((256, 262221),):
        case = synth.aneurysm_case(n, 0)
        dom = lbm.lbm_create_domain(case.mask, 0, lbm.LBM_F32, 0)
        assert lbm.lbm_fluid_count(dom) == expect == int((case.mask == synth.FLUID).sum())
        lbm.lbm_destroy(dom)


@pytest.mark.parametrize("bad", ["dims", "mask_value", "no_fluid", "periodic", "storage"])
def test_create_domain_rejects_bad_arguments(bad):
    lbm = _lbm()
    mask = np.ones((4, 5, 6), np.uint8)
    periodic, storage = 0, lbm.LBM_F32
    if bad == "dims":
        mask = np.ones((4, 5, 1100), np.uint8)
    elif bad == "mask_value":
        mask[1, 1, 1] = 7
    elif bad == "no_fluid":
        mask[...] = 0
    elif bad == "periodic":
        periodic = 9
    elif bad == "storage":
        storage = 11
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create_domain(mask, periodic, storage, 0)
    assert e.value.code == lbm.LBM_EINVAL


def test_parameter_validation_and_call_order():
    lbm = _lbm()
    case = synth.random_tiny_case(3)
    dom = lbm.lbm_create_domain(case.mask, case.periodic, lbm.LBM_F64, 0)
    try:
        for tau, s in ((0.5, (1, 1, 1, 1)), (0.8, (1, 2.0, 1, 1)), (0.8, (1, 0.0, 1, 1)),
                       (float("nan"), (1, 1, 1, 1))):
            with pytest.raises(lbm.LbmError) as e:
                lbm.lbm_set_params(dom, tau, s)
            assert e.value.code == lbm.LBM_EINVAL
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_set_params(dom, 0.8, (1, 1, 1, 1), (float("inf"), 0, 0))
        assert e.value.code == lbm.LBM_EINVAL
        lbm.lbm_set_params(dom, 0.8)
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_set_inlet_womersley(dom, (0, 0, 0), (1, 1, 1), 2.0, 1e-5, 1e-5, 0.01)
        assert e.value.code == lbm.LBM_EINVAL
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_set_inlet_womersley(dom, (0, 1, 0), (1, 1, 1), -1.0, 1e-5, 1e-5, 0.01)
        assert e.value.code == lbm.LBM_EINVAL
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_set_outlet_pressure(dom, 0.0)
        assert e.value.code == lbm.LBM_EINVAL
        # nothing attached yet: every call that needs device memory is out of order
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_init_equilibrium(dom)
        assert e.value.code == lbm.LBM_ESTATE
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_step(dom, 1)
        assert e.value.code == lbm.LBM_ESTATE
    finally:
        lbm.lbm_destroy(dom)


@pytest.mark.parametrize("maker", [lambda: synth.random_tiny_case(1, nx=11, ny=9, nz=8),
                                   lambda: synth.random_tiny_case(4, nx=31, ny=6, nz=5),
                                   lambda: synth.pipe_case(),
                                   lambda: synth.aneurysm_case(64, 2)])
def test_wall_links_match_an_independent_enumeration(maker):
    """lbm_wall_links lists the same (cell, direction) pairs, in the same
    order, as the seeded-input module's own enumeration from the mask."""
    lbm = _lbm()
    case = maker()
    got = lbm.lbm_wall_links(case.mask, case.periodic)
    ref = synth.wall_links(case.mask, case.periodic)
    assert got.shape == ref.shape and len(got) > 0
    assert np.array_equal(got, ref)


def test_curved_domain_validation_and_size():
    """Curved-wall links are checked one by one (EINVAL); a valid list turns
    the nodes that carry one into explicit-offset nodes, so the device
    footprint grows."""
    lbm = _lbm()
    case = synth.random_tiny_case(2, nx=11, ny=9, nz=8)
    links = synth.wall_links(case.mask, case.periodic)
    q = synth.random_wall_distances(links, 0)
    plain = lbm.lbm_create_domain(case.mask, case.periodic, lbm.LBM_F64, 0)
    curved = lbm.lbm_create_domain_curved(case.mask, case.periodic, lbm.LBM_F64, links, q, 0)
    assert lbm.lbm_device_bytes(curved) > lbm.lbm_device_bytes(plain)
    assert lbm.lbm_fluid_count(curved) == lbm.lbm_fluid_count(plain)
    lbm.lbm_destroy(plain)
    lbm.lbm_destroy(curved)
    fluid = np.argwhere(case.mask == synth.FLUID)[0]            # (z, y, x)
    notwall = None
    for a in range(27):
        cand = np.array([fluid[2], fluid[1], fluid[0], a], np.int32)
        if a != 13 and not any(np.array_equal(cand, l) for l in links):
            notwall = cand
            break
    solid = np.argwhere(case.mask == synth.SOLID)[0]
    bad_cases = [
        (links[:1], np.array([0.0])),                                   # q = 0
        (links[:1], np.array([1.5])),                                   # q > 1
        (links[:1], np.array([np.nan])),
        (np.concatenate([links[:1], links[:1]]), np.array([0.3, 0.4])),  # duplicate
        (np.array([[solid[2], solid[1], solid[0], links[0, 3]]], np.int32), np.array([0.3])),
        (np.array([[links[0, 0], links[0, 1], links[0, 2], 13]], np.int32), np.array([0.3])),
        (np.array([[99, 0, 0, 0]], np.int32), np.array([0.3])),
    ]
    if notwall is not None:
        bad_cases.append((notwall[None, :], np.array([0.3])))
    for lk, qq in bad_cases:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_create_domain_curved(case.mask, case.periodic, lbm.LBM_F64, lk, qq, 0)
        assert e.value.code == lbm.LBM_EINVAL


def test_streaming_mode_validation():
    """lbm_set_streaming takes its three modes before device memory is
    attached, also on a domain with curved walls; other values are EINVAL."""
    lbm = _lbm()
    case = synth.random_tiny_case(2, nx=11, ny=9, nz=8)
    plain = lbm.lbm_create_domain(case.mask, case.periodic, lbm.LBM_F32, 0)
    lbm.lbm_set_streaming(plain, "inplace")
    assert lbm.lbm_streaming_in_place(plain)
    lbm.lbm_set_streaming(plain, "pull")
    assert not lbm.lbm_streaming_in_place(plain)
    lbm.lbm_set_streaming(plain, "auto")
    assert not lbm.lbm_streaming_in_place(plain)   # a few kB of populations: pull
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_set_streaming(plain, 3)
    assert e.value.code == lbm.LBM_EINVAL
    links = synth.wall_links(case.mask, case.periodic)
    curved = lbm.lbm_create_domain_curved(case.mask, case.periodic, lbm.LBM_F32, links,
                                          synth.random_wall_distances(links, 0), 0)
    lbm.lbm_set_streaming(curved, "inplace")
    assert lbm.lbm_streaming_in_place(curved)
    lbm.lbm_set_streaming(curved, "pull")
    lbm.lbm_set_streaming(curved, "auto")
    assert not lbm.lbm_streaming_in_place(curved)
    lbm.lbm_destroy(plain)
    lbm.lbm_destroy(curved)


def test_streaming_auto_rule():
    """The automatic choice on the aneurysm geometries: in place for FP32 at
    400^3 and 512^3 (105 and 218 MiB per buffer) and FP64 at 400^3 (209 MiB);
    pull for FP64 at 512^3 (437 MiB per buffer), for every form at 256^3
    (the two buffers stay in the Infinity Cache) and for the 2-byte forms."""
    lbm = _lbm()
    expect = {512: {lbm.LBM_F32: True, lbm.LBM_F16S: False, lbm.LBM_BF16S: False, lbm.LBM_F64: False},
              400: {lbm.LBM_F32: True, lbm.LBM_F16S: False, lbm.LBM_F64: True},
              256: {lbm.LBM_F32: False, lbm.LBM_F16S: False, lbm.LBM_BF16S: False, lbm.LBM_F64: False}}
    for n, forms in expect.items():
        case = synth.aneurysm_case(n, 0)
        for storage, in_place in forms.items():
            dom = lbm.lbm_create_domain(case.mask, 0, storage, 0)
            assert lbm.lbm_streaming_in_place(dom) == in_place, (n, storage)
            lbm.lbm_destroy(dom)
        if n == 512:
            # curved walls step faster with pull: never in place by default
            links = synth.wall_links(case.mask, case.periodic)
            dom = lbm.lbm_create_domain_curved(case.mask, 0, lbm.LBM_F32, links, np.full(len(links), 0.3), 0)
            assert not lbm.lbm_streaming_in_place(dom)
            lbm.lbm_destroy(dom)


def test_probe_arguments_need_device_memory_and_fluid_cells():
    lbm = _lbm()
    case = synth.random_tiny_case(2, nx=11, ny=9, nz=8)
    dom = lbm.lbm_create_domain(case.mask, case.periodic, lbm.LBM_F64, 0)
    cnt = __import__("ctypes").c_int64(-1)
    lbm._check(lbm.load().lbm_probe_count(dom, __import__("ctypes").byref(cnt)))
    assert cnt.value == 0
    xyz = np.array([[0, 0, 0]], np.int32)
    rc = lbm.load().lbm_set_probes(dom, xyz.ctypes.data_as(lbm._P), 1, 1, lbm._P(64), 1)
    assert rc == lbm.LBM_ESTATE          # no device memory attached yet
    lbm.lbm_destroy(dom)


def test_unit_conversion_reproduces_the_papers_tau_pair():
    """Sec. 2.2.3 prints tau = 0.506 (dx 1e-4 m, dt 5e-6 s) and 0.503 (2e-4 m,
    1e-5 s).  Its stated nu = 3.2e-6 m^2/s gives 0.5048 instead; nu = 4e-6
    reproduces both printed values and the acoustic halving of tau - 1/2.  The
    quoted peak lattice speed 0.064 is 2.5 times the mean 0.512 m/s."""
    from paper_2101_11107_amd import units
    assert abs(units.lattice_tau(3.2e-6, 1e-4, 5e-6) - 0.5048) < 1e-12
    assert abs(units.lattice_tau(4.0e-6, 1e-4, 5e-6) - 0.506) < 1e-12
    assert abs(units.lattice_tau(4.0e-6, 2e-4, 1e-5) - 0.503) < 1e-12
    assert abs(units.acoustic_coarsen(0.506) - 0.503) < 1e-12
    assert abs(units.lattice_velocity(0.512, 1e-4, 5e-6) * 2.5 - 0.064) < 1e-12
    assert abs(units.fourier(4.0e-6, 2e-4, 1e-5) - 0.001) < 1e-15
    assert abs(units.physical_viscosity(0.506, 1e-4, 5e-6) - 4.0e-6) < 1e-18
