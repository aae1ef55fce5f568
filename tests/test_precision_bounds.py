"""Facts the FP32 parity bounds of the GPU tests rest on (CPU only, no method arithmetic)."""
import numpy as np

import workloads as W
from vrc_testutil import fp32_planes


def test_fp32_plane_shift_on_the_cylinder_mesh():
    """The FP32 walk of the 256^3 mesh of 0.2 cm voxels places plane k at lo + k h computed in FP32:
    against the FP64 planes a plane moves by at most 1.91e-6 cm and a voxel's width changes by at most
    1.53e-5 (the bound the cylinder precision test uses)."""
    wl = W.config3_precision(n_rays=0)
    for a, p32 in enumerate(fp32_planes(wl.mesh)):
        p64 = wl.mesh.lo[a] + np.arange(int(wl.mesh.n[a]) + 1) * wl.mesh.h[a]
        assert np.abs(p32 - p64).max() <= 1.91e-6
        assert np.abs(np.diff(p32) / np.diff(p64) - 1.0).max() <= 1.53e-5


def test_fp32_planes_exact_for_binary_spacings():
    """With lo and h FP32 numbers and k h exact (0.5 cm steps) the FP32 planes are the FP64 ones."""
    m = W.slab_mesh(1, 100, 0.5)
    for a, p in enumerate(fp32_planes(m)):
        np.testing.assert_array_equal(p, m.lo[a] + np.arange(101) * 0.5)
