"""Host-side check of the built library's gfx950 code objects (no GPU
needed): no kernel keeps private scratch memory except the ones listed
here.  A kernel that spills to scratch pays for it on every launch (the
dense neighbour query once grew from 4 to 70 microseconds per launch on
frames without dense rows, where it only tests each segment, when a
second inlined copy of its search took it past its register budget)."""
import os
import re
import shutil
import struct
import subprocess

import pytest

# kernel -> largest private segment (bytes per lane) it may keep: the
# adjoint holds a track's state, its adjoint and the tape addresses in FP64
# at 256 VGPRs and spills the rest
ALLOWED = {"adj_tracks": 176}

READELF = next((p for p in ("/opt/rocm/llvm/bin/llvm-readelf", shutil.which("llvm-readelf"))
                if p and os.path.exists(p)), None)


def _section(data, wanted):
    """Bytes of ELF64 section `wanted` of a little-endian shared object."""
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)

    def header(i):
        return struct.unpack_from("<IIQQQQIIQQ", data, shoff + i * shentsize)

    names = header(shstrndx)
    for i in range(shnum):
        h = header(i)
        raw = data[names[4] + h[0]:]
        if raw[:raw.index(b"\0")].decode() == wanted:
            return data[h[4]:h[4] + h[5]]
    return None


def _gfx950_objects(fatbin):
    """Device code objects of the offload bundles in the fat binary (one
    bundle per translation unit): header magic, entry count, then per entry
    its offset, size and target id."""
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    objs, pos = [], 0
    while (p := fatbin.find(magic, pos)) >= 0:
        n, = struct.unpack_from("<Q", fatbin, p + len(magic))
        q = p + len(magic) + 8
        for _ in range(n):
            off, size, idlen = struct.unpack_from("<QQQ", fatbin, q)
            q += 24
            ident = fatbin[q:q + idlen].decode()
            q += idlen
            if "gfx950" in ident:
                objs.append(fatbin[p + off:p + off + size])
        pos = p + len(magic)
    return objs


def _kernels(readelf_notes):
    """(name, private segment bytes, VGPR spills) per kernel of the YAML
    metadata that llvm-readelf prints (kernel keys sit at four spaces)."""
    out = []
    for block in re.split(r"^  - (?=\.)", readelf_notes, flags=re.M)[1:]:
        block = "    " + block
        name = re.search(r"^    \.name:\s+(\S+)", block, re.M).group(1)
        priv = int(re.search(r"^    \.private_segment_fixed_size:\s+(\d+)", block, re.M).group(1))
        spill = re.search(r"^    \.vgpr_spill_count:\s+(\d+)", block, re.M)
        out.append((name, priv, int(spill.group(1)) if spill else 0))
    return out


@pytest.mark.skipif(READELF is None, reason="llvm-readelf not found")
def test_no_kernel_spills_to_scratch(tmp_path):
    from paper_2412_13755_amd import _capi
    data = open(_capi.LIB_PATH, "rb").read()
    fat = _section(data, ".hip_fatbin")
    assert fat is not None, "no .hip_fatbin section"
    objs = _gfx950_objects(fat)
    assert objs, "no gfx950 code object"
    kernels = []
    for k, obj in enumerate(objs):
        f = tmp_path / ("co%d.elf" % k)
        f.write_bytes(obj)
        notes = subprocess.run([READELF, "--notes", str(f)], capture_output=True, text=True,
                               check=True).stdout
        kernels += _kernels(notes)
    assert len(kernels) > 50
    names = [n for n, _, _ in kernels]
    assert any("nb_query_dense" in n for n in names)
    bad = []
    for name, priv, spill in kernels:
        limit = next((v for k, v in ALLOWED.items() if k in name), 0)
        if priv > limit:
            bad.append((name, priv, spill))
    assert not bad, "kernels with private scratch (bytes per lane, VGPR spills): %r" % bad
