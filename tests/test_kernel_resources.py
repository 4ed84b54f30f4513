"""The hot kernels keep the occupancy their design relies on (CPU only).

build() collects the compiler's per-kernel resource report (registers, LDS,
spills, waves per SIMD) into paper_2304_12557_amd/kernel_resources.json.  A
kernel that silently drops to one wave per SIMD halves its latency hiding:
that happened to the 3-D decompression kernel (256 VGPRs plus 2 AGPRs), and
its 512^3 time went from 132 to 152 us.  So:

* the compression kernels (per-field and batched) run 2 workgroups of 4 waves
  per CU: 2 waves per SIMD and at most 80 KB of LDS per workgroup;
* every decompression kernel (both per-field forms, fp64 output, integer
  output, batched) runs 2 waves per SIMD without spilling to scratch;
* the range pass, a plain streaming read, runs at least 4 waves per SIMD.
"""
import json
import os

import pytest

PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2304_12557_amd",
                    "kernel_resources.json")


@pytest.fixture(scope="module")
def res():
    if not os.path.exists(PATH):
        pytest.skip("no kernel resource report: run build() first")
    with open(PATH) as fh:
        return json.load(fh)


def family(res, prefix):
    out = {k: v for k, v in res.items() if k.startswith(prefix)}
    assert out, prefix
    return out


# the per-field kernel: 3 ranks x (16-byte loads, or one load per value for a
# misaligned pointer) x 2 fp32 quantizers, plus 3 ranks on the integers of the
# fp64 and field-global paths (always 16-byte loads); the batched one: 3 ranks
# x 2 load widths
@pytest.mark.parametrize("prefix,count", [("_ZN2fz10k_compressI", 15), ("_ZN2fz16k_batch_compressI", 6)])
def test_compression_two_workgroups_per_cu(res, prefix, count):
    ks = family(res, prefix)
    assert len(ks) == count, sorted(ks)
    for k, v in ks.items():
        assert v["waves_per_simd"] >= 2, (k, v)
        assert v["lds_bytes"] <= 80 * 1024, (k, v)


@pytest.mark.parametrize("prefix,count", [("_ZN2fz12k_decompressI", 6), ("_ZN2fz18k_decompress_splitI", 6),
                                          ("_ZN2fz14k_decompress64I", 6), ("_ZN2fz16k_decompress_intI", 6),
                                          ("_ZN2fz18k_batch_decompress", 1)])
def test_decompression_two_waves_per_simd_no_spill(res, prefix, count):
    ks = family(res, prefix)
    assert len(ks) == count, sorted(ks)
    for k, v in ks.items():
        assert v["waves_per_simd"] >= 2, (k, v)
        assert v["agprs"] == 0 and v["vgprs"] + v["agprs"] <= 256, (k, v)
        assert v["scratch_bytes_per_lane"] == 0 and v["vgpr_spills"] == 0, (k, v)


def test_range_pass_streams(res):
    for k, v in family(res, "_ZN2fz8k_minmax").items():
        assert v["waves_per_simd"] >= 4, (k, v)
