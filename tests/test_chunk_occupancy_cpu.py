"""The chunk kernel's occupancy, read from the gfx950 assembly of the library
(no GPU needed): its speed follows the one-wave workgroups each SIMD holds
(five instead of six per SIMD cost 8% on the 4 Gbase build), so its LDS and
registers are held to budgets. Occupancy on gfx950: 512 vector registers per
lane of a SIMD, allocated in granules of 8; 160 KB of LDS per CU, counted
here in granules of 512 bytes; four SIMDs per CU."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1401_7457_amd import build as pkg_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc is not installed")
    out = tmp_path_factory.mktemp("asm") / "cxbwt.s"
    flags = [f for f in pkg_build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "paper_1401_7457_amd", "csrc", "cxbwt.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    text = out.read_text()
    found = {}
    for m in re.finditer(r"\.amdhsa_kernel (\S+)\n(.*?)\.end_amdhsa_kernel", text, re.S):
        body = m.group(2)
        field = lambda k: int(re.search(rf"\.amdhsa_{k} (\d+)", body).group(1))
        found[m.group(1)] = {"lds": field("group_segment_fixed_size"), "scratch": field("private_segment_fixed_size"),
                             "vgpr": field("next_free_vgpr")}
    return found


def chunk_kernel(kernels, li, persistent=False):
    pat = re.compile(rf"k_localILi{li}ELi\d+ELb{1 if persistent else 0}E")
    hits = [v for k, v in kernels.items() if pat.search(k)]
    assert len(hits) == 1, f"one chunk kernel with {li} suffixes a lane (persistent={persistent})"
    return hits[0]


def waves_per_simd(k):
    by_regs = 512 // (-(-k["vgpr"] // 8) * 8)
    by_lds = 163840 // (-(-k["lds"] // 512) * 512) // 4  # one wave per workgroup
    return min(by_regs, by_lds, 8)


def test_384_suffix_chunks_keep_six_waves_per_simd(kernels):
    k = chunk_kernel(kernels, 6)
    assert k["scratch"] == 0
    assert k["lds"] <= 163840 // 24, k
    assert waves_per_simd(k) >= 6, k


def test_512_and_192_suffix_chunks(kernels):
    k8, k3 = chunk_kernel(kernels, 8), chunk_kernel(kernels, 3)
    assert k8["scratch"] == 0 and k3["scratch"] == 0
    assert waves_per_simd(k8) >= 4, k8
    assert waves_per_simd(k3) >= 7, k3


def test_chunk_lds_follows_the_chunk_size(kernels):
    # per suffix: key 8 B, handle 4 B, live-list entry and group number 2 B
    # each, half a group-table entry 1 B, a head bit: 17.1 B (the split
    # counters, 1 KB, share the list's space)
    for li in (3, 6, 8):
        k = chunk_kernel(kernels, li)
        assert 17 * 64 * li <= k["lds"] <= 17.5 * 64 * li, (li, k)
