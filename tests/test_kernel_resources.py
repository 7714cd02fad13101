"""Resource budget of the shooting kernel's default instances, read from the
metadata of the gfx950 code object inside the built liblensmap.so (no GPU).

The FP32 table path is issue-bound and needs 4 waves per SIMD to hide its LDS
and reciprocal latencies: 256-thread workgroups, 4 per CU, so at most 128
VGPRs (no AGPRs) and 40 KiB of LDS per workgroup, no register spills to
scratch memory.  A change that crosses the VGPR line drops occupancy to 3
waves per SIMD and costs more than 10% of the shooting rate."""
import os

import pytest

import paper_2308_14278_amd.lensmap as lm
from paper_2308_14278_amd import codeobj

# <scheme 1 (interpolated), precision 0 (mixed) or 4 (centred), NR, P 4, LDS layout>; the
# batch kernel must fit without spills in every LDS layout the tuner may pick,
# the per-map kernel (descriptor by value, held to 4 waves by an attribute) may
# spill a few per-unit values to scratch
BATCH = "_ZN12_GLOBAL__N_113k_shoot_batchILi1ELi%dELi%dELi4ELi%dEEEvPK6LmDescPKlPKiiPy"
DEFAULT = tuple([(BATCH % (0, nr, lay), 0) for nr in (8, 16) for lay in range(4)] +
                # the centred sums (the default on the paper's own map) at 8 rays per
                # lane, in the one LDS layout they are built for
                [(BATCH % (4, 8, 0), 0)] +
                [("_ZN12_GLOBAL__N_111k_shoot_mapILi1ELi0ELi16ELi4EEEv6LmDesc", 4),
                 # the plain FP32 comparison path (precision 1), per map and batched
                 ("_ZN12_GLOBAL__N_111k_shoot_mapILi1ELi1ELi16ELi4EEEv6LmDesc", 4),
                 (BATCH % (1, 16, 0), 0)])


def test_default_shooting_kernels_fit_four_waves_per_simd():
    if not codeobj.tools_available():
        pytest.skip("ROCm LLVM tools not found")
    if not os.path.exists(lm.LIB_PATH):
        pytest.fail("liblensmap.so is not built")
    kernels = codeobj.kernel_metadata()
    for name, max_spill in DEFAULT:
        assert name in kernels, "kernel %s not in the code object" % name
        k = kernels[name]
        print("%s: %s VGPRs (%s spilled), %s AGPRs, %s B LDS, %s SGPR spills" % (
            name, k["vgpr_count"], k["vgpr_spill_count"], k["agpr_count"],
            k["group_segment_fixed_size"], k["sgpr_spill_count"]))
        assert int(k["vgpr_count"]) + int(k["agpr_count"]) <= 128
        assert int(k["vgpr_spill_count"]) <= max_spill
        assert int(k["private_segment_fixed_size"]) <= 4 * max_spill
        assert int(k["group_segment_fixed_size"]) <= 40 * 1024
        assert int(k["max_flat_workgroup_size"]) == 256


def test_kernel_code_hash_is_a_function_of_the_code():
    """The per-kernel machine-code hash that keys the traffic measurements: two
    reads of the same library agree, and distinct kernels hash apart."""
    if not codeobj.tools_available():
        pytest.skip("ROCm LLVM tools not found")
    a = codeobj.kernel_code_sha(BATCH % (0, 16, 0))
    assert a is not None and len(a) == 16
    assert codeobj.kernel_code_sha(BATCH % (0, 16, 0)) == a
    assert codeobj.kernel_code_sha(BATCH % (0, 16, 1)) not in (None, a)
    assert codeobj.kernel_code_sha("no_such_kernel") is None
