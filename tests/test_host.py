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
