"""Resource checks on the compiled gfx950 kernels (host only: hipcc cross-compiles).

The triangle kernel is register-tight (two waves per SIMD, up to 160 int32
accumulators per lane): it must compile without scratch, since spill traffic in
its stage loop would stall it on memory, and its staging and operand buffers
must fit the 160 KiB of LDS of a gfx950 compute unit."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1503_06203_amd", "csrc")


def device_asm(src, tmp_path):
    from paper_1503_06203_amd import build
    out = tmp_path / "k.s"
    cmd = [build.HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "--cuda-device-only", "-S",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, src), "-o", str(out)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        pytest.skip("hipcc unavailable: " + res.stderr[-300:])
    return out.read_text()


def kernel_field(asm, kernel, field):
    # the .amdhsa_kernel block of the kernel holds its resource fields
    m = re.search(r"\.amdhsa_kernel\s+\S*%s\S*(.*?)\.end_amdhsa_kernel" % kernel, asm, re.S)
    assert m, kernel
    f = re.search(r"\.%s\s+(\d+)" % field, m.group(1))
    assert f, field
    return int(f.group(1))


def test_triangle_kernel_has_no_scratch_and_fits_lds(tmp_path):
    asm = device_asm("xcorr_tri.hip", tmp_path)
    for kernel in ("xcorr_tri_kernel", "xcorr_tri_delay_kernel", "xcorr_tri_window_kernel",
                   "xcorr_tri_segments_kernel"):
        assert kernel_field(asm, kernel, "amdhsa_private_segment_fixed_size") == 0
    for kernel in ("xcorr_tri_kernel", "xcorr_tri_delay_kernel", "xcorr_tri_window_kernel",
                   "xcorr_tri_segments_kernel"):
        assert kernel_field(asm, kernel, "amdhsa_group_segment_fixed_size") <= 160 * 1024


def test_bf6_triangle_kernel_has_no_scratch_and_fits_lds(tmp_path):
    # spills here would also add scratch loads to the vector-memory queue the
    # staging waits count on (correct, but each wait would then cover them too)
    asm = device_asm("xcorr_tri_bf6.hip", tmp_path)
    assert kernel_field(asm, "xcorr_tri_bf6_kernel", "amdhsa_private_segment_fixed_size") == 0
    assert kernel_field(asm, "xcorr_tri_bf6_kernel", "amdhsa_group_segment_fixed_size") <= 160 * 1024


def test_rect_kernel_has_no_scratch_and_fits_lds(tmp_path):
    # the kernel for n > 256 (diagonal squares and off-diagonal tiles): two
    # waves per SIMD with 128-160 accumulators each; a spill would put scratch
    # traffic into the vector-memory queue that the staging waits count on
    # (and its persistent queue form, which runs the same pieces per queue item)
    asm = device_asm("xcorr_rect.hip", tmp_path)
    for kernel in ("xcorr_rect_kernel", "xcorr_rect_segments_kernel", "xcorr_queue_kernel"):
        assert kernel_field(asm, kernel, "amdhsa_private_segment_fixed_size") == 0, kernel
        assert kernel_field(asm, kernel, "amdhsa_group_segment_fixed_size") <= 160 * 1024, kernel


def test_rect_bf6_kernel_has_no_scratch_and_fits_lds(tmp_path):
    # 128 fp32 accumulators and bf6 operands (8-register tuples) per wave: the
    # decode and the MFMA segments are kept apart so that they fit
    asm = device_asm("xcorr_rect_bf6.hip", tmp_path)
    assert kernel_field(asm, "xcorr_rect_bf6_kernel", "amdhsa_private_segment_fixed_size") == 0
    assert kernel_field(asm, "xcorr_rect_bf6_kernel", "amdhsa_group_segment_fixed_size") <= 160 * 1024


def test_small_kernel_has_no_scratch_and_fits_lds(tmp_path):
    # each wave waits on a count of its own outstanding loads; scratch
    # traffic would join that queue
    asm = device_asm("xcorr_small.hip", tmp_path)
    assert kernel_field(asm, "xcorr_small_kernel", "amdhsa_private_segment_fixed_size") == 0
    assert kernel_field(asm, "xcorr_small_kernel", "amdhsa_group_segment_fixed_size") <= 160 * 1024


def test_shift_and_tile_kernels_have_no_scratch_and_fit_lds(tmp_path):
    # the delay shift's loader waves wait on a count of their own loads, and
    # the general tile kernel holds 128 accumulators per lane: neither may spill
    asm = device_asm("xcorr_shift.hip", tmp_path)
    assert kernel_field(asm, "xcorr_shift_kernel", "amdhsa_private_segment_fixed_size") == 0
    assert kernel_field(asm, "xcorr_shift_kernel", "amdhsa_group_segment_fixed_size") <= 160 * 1024
    asm = device_asm("xcorr_tile.hip", tmp_path)
    blocks = re.findall(r"\.amdhsa_kernel\s+(\S*xcorr_tile128_kernel\S*)", asm)
    assert len(blocks) == 2, blocks   # dword-aligned and byte-wise loads
    for name in blocks:
        assert kernel_field(asm, re.escape(name), "amdhsa_private_segment_fixed_size") == 0, name
        assert kernel_field(asm, re.escape(name), "amdhsa_group_segment_fixed_size") <= 160 * 1024
