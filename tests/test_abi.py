"""The C-ABI library loads and exports every function the public headers
declare; host-side argument checks that need no GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")

DECL = re.compile(r"^\s*(?:const\s+)?(?:int|void|char|double|size_t|int64_t)\s*\*?\s*(lbm\w+)\s*\(", re.M)


def _declared():
    names = []
    for fn in sorted(os.listdir(INCLUDE)):
        if fn.endswith(".h"):
            with open(os.path.join(INCLUDE, fn)) as f:
                names += DECL.findall(f.read())
    return names


def test_headers_declare_functions():
    names = _declared()
    assert "lbm_step" in names and "lbmnet_forward" in names and "lbm_batch_step" in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2101_11107_amd import lbm
    lib = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared function under the same name
    assert sorted(set(_declared())) == sorted(set(lbm.EXPORTED))
    lbm.load()


def test_network_table_matches_oracle():
    from oracle import o3_net as o3
    from paper_2101_11107_amd import net as nn
    assert nn.lbmnet_param_count() == sum(co * 27 * ci + co for _, ci, co, _, _ in o3.LAYERS)
    levels = {"c": 0, "h": 1, "f": 2}
    for (name, ci, co, relu, lev), row in zip(o3.LAYERS, nn.layer_table()):
        assert row[:5] == (name, ci, co, int(relu), levels[lev])


def test_network_argument_checks():
    from paper_2101_11107_amd import lbm
    from paper_2101_11107_amd import net as nn
    for dims in ((1, 3, 4, 32), (1, 4, 4, 48), (0, 4, 4, 32), (1, 4, 4, 16)):
        with pytest.raises(lbm.LbmError) as e:
            nn.lbmnet_create(*dims, 1, 0)
        assert e.value.code == lbm.LBM_EINVAL
    h = nn.lbmnet_create(2, 4, 4, 32, 1, 0)
    ht = nn.lbmnet_create(2, 4, 4, 32, 0, 0)
    assert nn.lbmnet_device_bytes(h) > nn.lbmnet_device_bytes(ht) > 0
    assert nn.lbmnet_adam_count(h) == 0
    nn.lbmnet_destroy(h)
    nn.lbmnet_destroy(ht)
    for bad in ((1, 2, 2, 16, 3, 4), (1, 2, 2, 8, 4, 4), (1, 2, 2, 16, 4, 36)):
        with pytest.raises(lbm.LbmError) as e:
            nn.lbmnet_conv3d_workspace(*bad)
        assert e.value.code == lbm.LBM_EINVAL
    assert nn.lbmnet_conv3d_workspace(1, 2, 2, 16, 4, 4) > 0


def test_library_womersley_profile_matches_closed_form():
    """The library's host-side Womersley profile (its own complex J0 series)
    against the closed form evaluated with scipy's Bessel function (the
    oracle's definition), across radii, phases and Womersley numbers 1-8."""
    import math
    import numpy as np
    from oracle import o1_dense as o1
    from paper_2101_11107_amd import lbm
    R = 12.0
    for alpha in (1.0, 3.0, 8.0):
        omega = 2 * math.pi / 4000.0
        nu = omega * R * R / alpha ** 2
        G0 = 4 * nu * 0.0329 / (R * R)
        for t in (0.0, 517.0, 1999.0, 3333.0):
            rs = np.array([0.0, 1.5, 6.0, 11.0, 11.99, 12.0, 13.0])
            ref = o1.womersley_speed(rs, t, R, nu, G0, G0, omega)
            got = np.array([lbm.lbm_inlet_profile(r, t, R, nu, G0, G0, omega) for r in rs])
            assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)) + 1e-18, (alpha, t)
    # omega = 0: steady Poiseuille
    assert abs(lbm.lbm_inlet_profile(3.0, 0.0, R, 0.02, 1e-6, 0.0, 0.0) - 1e-6 * (R * R - 9.0) / 0.08) < 1e-15


def test_noalloc_layer_rejects_workspace_beyond_its_fixed_array():
    """lbmnet_conv3d_noalloc refuses, before touching the GPU, a layer whose
    workspace exceeds the library's fixed array, and reports that size."""
    from paper_2101_11107_amd import lbm
    from paper_2101_11107_amd import net as nn
    limit = nn.lbmnet_conv3d_noalloc_limit()
    assert limit == 64 << 20
    dims = (4, 64, 64, 128, 32, 32)
    assert nn.lbmnet_conv3d_workspace(*dims) > limit
    with pytest.raises(lbm.LbmError) as e:
        nn.lbmnet_conv3d_noalloc(*dims, 1, *[None] * 8, 0)
    assert e.value.code == lbm.LBM_EINVAL
    assert "workspace" in str(e.value)
    with pytest.raises(lbm.LbmError) as e:
        nn.lbmnet_conv3d_noalloc(1, 3, 4, 16, 5, 16, 1, *[None] * 8, 0)   # cin not a multiple of 4
    assert e.value.code == lbm.LBM_EINVAL
