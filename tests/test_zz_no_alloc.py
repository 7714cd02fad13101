"""The allocation-free entry point lm_peak_stats_noalloc against lm_peak_stats
(which allocates its device staging), through the C ABI: equal results on
two calls in a row, the second with fewer rows, fewer bins and other edges
(the scratch memory keeps the first call's contents), and its size limits."""
import numpy as np
import pytest

import paper_2308_14278_amd.lensmap as lm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    lm.load()


def _fold_map():
    import math
    k0, dx, dy, ks = 0.83, 2.0e-3, -1.5e-3, 0.01
    g = lm.lm_geometry_derive_fold(4.0, 4.0, 500, 300, k0, dx, ks, n_rays=3e7, coarse=64)
    hx, hy = g.ray_nx * g.ray_dx / 2, g.ray_ny * g.ray_dy / 2
    n = int(round(4 * hx * hy * ks / math.pi))
    rng = np.random.default_rng(77)
    x, y = rng.uniform(-hx, hx, n), rng.uniform(-hy, hy, n)
    mp = lm.Map(g, kappa_star=ks, lenses=(x, y, np.ones(n)), fold=(k0, dx, dy))
    mp.shoot()
    return g, mp


def test_noalloc_matches_allocating_entry_point():
    g, mp = _fold_map()
    x0, x1 = g.src_x0, g.src_x0 + g.src_nx * g.src_dx
    calls = [(list(range(5, 295, 7)), np.linspace(x0, x1, 40), 5),
             (list(range(100, 140, 9)), np.linspace(x0 + 0.3, x1 - 1.0, 9), 4)]
    total = 0
    for tracks, edges, k in calls:
        want = lm.lm_peak_stats(mp.h, tracks, edges, k)
        got = lm.lm_peak_stats_noalloc(mp.h, tracks, edges, k)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
        total += int(want[0].sum())
    print("true peaks over both calls: %d" % total)
    assert total > 0
    # the first call's larger tables left in scratch do not leak into a smaller call
    again = lm.lm_peak_stats_noalloc(mp.h, *calls[1][:2], calls[1][2])
    for a, b in zip(again, lm.lm_peak_stats(mp.h, *calls[1][:2], calls[1][2])):
        np.testing.assert_array_equal(a, b)
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_peak_stats_noalloc(mp.h, [1] * 8193, np.linspace(x0, x1, 3))
    assert e.value.status == lm.LM_EINVAL
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_peak_stats_noalloc(mp.h, [1], np.linspace(x0, x1, 4098))
    assert e.value.status == lm.LM_EINVAL
    mp.close()
