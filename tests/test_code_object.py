"""Resource check of the built library's gfx950 code objects (CPU only).

The resident kernels keep a member's whole state in registers, and their
co-resident capacity (how many slice pairs one launch holds) depends on the
register count the compiler lands on: every variant except the one-wave
192x192 ones and the 8 x 8 x 4 plan at 256x256 must fit two waves per SIMD,
i.e. at most 256 VGPRs + AGPRs per lane.  One compiler run put the 16 x 256 variant at 257
registers, which halved the pairs it holds; this test reads the kernel
metadata of the library built here (llvm-objcopy, clang-offload-bundler's
bundle format, llvm-readelf --notes) and fails on such a drift.
"""
import os
import re
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2006_09808_amd", "libpd_hip.so")
LLVM = "/opt/rocm/llvm/bin"


def _kernel_registers(tmp_path):
    """{kernel symbol: (vgpr_count, agpr_count)} of every gfx950 kernel."""
    objcopy, readelf = os.path.join(LLVM, "llvm-objcopy"), os.path.join(LLVM, "llvm-readelf")
    if not (os.path.exists(LIB) and os.path.exists(objcopy) and os.path.exists(readelf)):
        pytest.skip("library not built or ROCm LLVM tools missing")
    fatbin = str(tmp_path / "pd.fatbin")
    subprocess.run([objcopy, "--dump-section", ".hip_fatbin=" + fatbin, LIB, str(tmp_path / "copy.so")],
                   check=True, capture_output=True)
    data = open(fatbin, "rb").read()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    regs = {}
    for k, st in enumerate(m.start() for m in re.finditer(re.escape(magic), data)):
        n = struct.unpack_from("<Q", data, st + len(magic))[0]
        p = st + len(magic) + 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", data, p)
            p += 24
            triple = data[p:p + tlen].decode()
            p += tlen
            if not triple.endswith("gfx950"):
                continue
            co = tmp_path / ("co%d.o" % k)
            co.write_bytes(data[st + off:st + off + size])
            notes = subprocess.run([readelf, "--notes", str(co)], check=True, capture_output=True,
                                   text=True).stdout
            for blk in notes.split("  - .agpr_count")[1:]:
                blk = ".agpr_count" + blk
                name = re.search(r"\.name:\s+(\S+)", blk)
                vg = re.search(r"\.vgpr_count:\s+(\d+)", blk)
                ag = re.search(r"\.agpr_count:\s+(\d+)", blk)
                if name and vg and ag:
                    regs[name.group(1)] = (int(vg.group(1)), int(ag.group(1)))
    return regs


def test_resident_kernels_fit_two_waves_per_simd(tmp_path):
    regs = _kernel_registers(tmp_path)
    res = {k: v for k, v in regs.items() if "k_resident" in k}
    # the bench's kernel and the other default-plan 256x256 variants are there
    assert any("k_residentILi256ELi256ELi8ELi512ELi0E" in k for k in res)
    assert len(res) >= 15, sorted(res)
    # one wave per SIMD by design: the 192x192 variants without a waves
    # argument (their two-wave twins, ...ELi2EEE, are checked) and the
    # 8 x 8 x 4 plan at 256x256
    one_wave = ("ILi192ELi192ELi12ELi256ELi0ELi0E", "ILi192ELi192ELi24ELi128ELi0ELi0E",
                "ILi256ELi256ELi16ELi256ELi1E")
    assert any("ILi192ELi192ELi12ELi256ELi0ELi2E" in k for k in res)
    for k, (vgpr, agpr) in sorted(res.items()):
        if any(t in k for t in one_wave):
            continue
        # .vgpr_count counts the unified file (AGPRs included) on gfx950
        assert vgpr <= 256, "%s: %d registers (%d AGPRs): below two waves per SIMD" % (k, vgpr, agpr)
