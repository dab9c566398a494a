"""The gfx950 code objects inside the built library contain no packed-FP32
arithmetic (v_pk_add_f32 / v_pk_mul_f32 / v_pk_fma_f32).  Those instructions
are kept out by the build (packed-FP32 instruction selection is disabled), and
this test disassembles what was actually built to hold it to that.  CPU only:
it reads the library's offload bundles, no device is needed."""
import os
import re
import struct
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2505_08985_amd", "libpndf.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
PACKED_F32 = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


def code_objects(fatbin):
    """Split the .hip_fatbin section into its gfx950 ELF code objects.  The
    section is a run of uncompressed clang offload bundles: magic, entry count,
    then per entry (offset, size, id length, id), offsets relative to the bundle."""
    out, pos = [], 0
    while True:
        pos = fatbin.find(MAGIC, pos)
        if pos < 0:
            return out
        p = pos + len(MAGIC)
        (n,) = struct.unpack_from("<Q", fatbin, p)
        p += 8
        for _ in range(n):
            off, size, idlen = struct.unpack_from("<QQQ", fatbin, p)
            p += 24
            ident = fatbin[p:p + idlen].decode()
            p += idlen
            if "gfx950" in ident and size:
                out.append((ident, fatbin[pos + off:pos + off + size]))
        pos = p


@pytest.fixture(scope="module")
def disassembly():
    if not os.path.exists(LIB):
        import paper_2505_08985_amd.build as b
        b.build()
    for tool in ("llvm-objcopy", "llvm-objdump"):
        if not os.path.exists(os.path.join(LLVM, tool)):
            pytest.skip("%s not installed" % tool)
    with tempfile.TemporaryDirectory() as d:
        fb = os.path.join(d, "fatbin")
        subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", ".hip_fatbin=" + fb,
                        LIB, os.path.join(d, "stripped")], check=True)
        objs = code_objects(open(fb, "rb").read())
        texts = []
        for k, (ident, blob) in enumerate(objs):
            path = os.path.join(d, "co%d" % k)
            open(path, "wb").write(blob)
            r = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", path],
                               check=True, stdout=subprocess.PIPE, text=True)
            texts.append(r.stdout)
    return texts


def test_every_device_source_has_a_gfx950_code_object(disassembly):
    # mesh, hier, eval, sample, projarea (and any host source that carries device code)
    assert len(disassembly) >= 5
    joined = "\n".join(disassembly)
    for kernel in ("k_build_mesh", "k_level1", "k_eval_plain", "k_sample", "k_projected_area"):
        assert kernel in joined, kernel


def test_no_packed_fp32_arithmetic(disassembly):
    hits = []
    for text in disassembly:
        hits += [l.strip() for l in text.splitlines() if PACKED_F32.search(l)]
    assert not hits, "packed FP32 instructions in the gfx950 code: %s" % hits[:5]


def test_disassembly_sees_packed_instructions_when_present(disassembly):
    """The scan is not vacuous: packed forms are disassembled by name, e.g. the
    packed 16-bit integer max/min the traversal's box test uses on purpose."""
    assert PACKED_F32.search("  v_pk_fma_f32 v[0:1], v[2:3], v[4:5], v[6:7]")
    joined = "\n".join(disassembly)
    assert re.search(r"\bv_pk_(max|min)_u16\b", joined)
