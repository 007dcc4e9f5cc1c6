"""GPU parity of the snow-cover node (section 5.1) through the C ABI against the CPU oracle: the alpha
raster is bit-exact (the same binary32 ramps in the same order) on ragged grids, with and without blend
zones, at the full 2048^2 alpine tile, and with an output that is not 16-byte aligned (the kernel's
scalar path)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def avl():
    import paper_2506_23364_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [
    ("ragged_67x45", 67, 45, (0.4, 120.0, 42.0, 10.0)),
    ("steps_only", 50, 51, (0.5, 0.0, 35.0, 0.0)),
    ("wide_blend", 33, 97, (0.2, 900.0, 70.0, 60.0)),
    ("tiny_3x1", 3, 1, (0.5, 10.0, 40.0, 5.0)),
]


@pytest.mark.parametrize("name,h,w,p", CASES, ids=[c[0] for c in CASES])
def test_snow_cover_bit_exact(avl, name, h, w, p):
    dem = synth.alpine_dem(max(h, w, 2), 1500.0, seed=h * 7 + w)[:h, :w].copy()
    q, zb, smax, sb = p
    line = float(np.quantile(dem, q))
    if min(h, w) >= 2:
        nrm_ref = oracle.normals(dem, 10.0)
        nrm = avl.normals(dev(dem), 10.0)
    else:
        rng = np.random.default_rng(1)
        nrm_ref = np.zeros((h, w, 4), np.float32)
        nrm_ref[..., 2] = rng.uniform(0.5, 1.0, (h, w))
        nrm = dev(nrm_ref)
    ref = oracle.snow_cover(nrm_ref, dem, line, zb, smax, sb)
    got = avl.snow_cover(nrm, dev(dem), line, zb, smax, sb).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), np.argwhere(got != ref)[:5]


def test_snow_cover_alpine_full_size(avl):
    w = synth.make_workload("alpine")
    dem = w.dem
    nrm = avl.normals(dev(dem), w.cell_size)
    ref = oracle.snow_cover(oracle.normals(dem, w.cell_size), dem, 1400.0, 250.0, 40.0, 8.0)
    got = avl.snow_cover(nrm, dev(dem), 1400.0, 250.0, 40.0, 8.0).cpu().numpy()
    assert 0 < (ref > 0).mean() < 1 and ((ref > 0) & (ref < 1)).any()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_snow_cover_unaligned_output(avl):
    dem = synth.alpine_dem(40, 800.0, seed=2)[:37, :39].copy()
    h, w = dem.shape
    nrm = avl.normals(dev(dem), 10.0)
    ref = oracle.snow_cover(oracle.normals(dem, 10.0), dem, float(np.median(dem)), 50.0, 45.0, 10.0)
    buf = torch.full((h * w + 1,), -1.0, dtype=torch.float32, device="cuda")
    d = dev(dem)
    rc = avl.lib.avl_snow_cover(nrm.data_ptr(), d.data_ptr(), h, w, float(np.median(dem)), 50.0, 45.0, 10.0,
                                buf.data_ptr() + 4, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    got = buf.cpu().numpy()
    assert got[0] == -1.0
    assert np.array_equal(got[1:].reshape(h, w).view(np.uint32), ref.view(np.uint32))
