"""Device code of the built library, read back as gfx950 assembly.

The HIP objects keep their device code in a `.hip_fatbin` section: one
clang offload bundle per compiled source, each holding a host entry (empty)
and a gfx950 code object.  This module finds that section with a minimal
ELF64 reader, splits the bundles, and disassembles the gfx950 code objects
with the ROCm llvm-objdump.  It reads only code built here, from the
repository's own sources."""
import os
import re
import struct
import subprocess
import tempfile

OBJDUMP = os.environ.get("FDBB_OBJDUMP", "/opt/rocm/llvm/bin/llvm-objdump")
BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def elf_section(path: str, name: str) -> bytes:
    """Bytes of the named section of a little-endian ELF64 file."""
    data = open(path, "rb").read()
    if data[:4] != b"\x7fELF" or data[4] != 2 or data[5] != 1:
        raise ValueError(f"{path}: not a little-endian ELF64 file")
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)

    def header(k):
        off = shoff + k * shentsize
        sh_name, sh_type, _flags, _addr, sh_offset, sh_size = struct.unpack_from("<IIQQQQ", data, off)
        return sh_name, sh_type, sh_offset, sh_size

    _, _, str_off, str_size = header(shstrndx)
    names = data[str_off:str_off + str_size]
    for k in range(shnum):
        sh_name, sh_type, off, size = header(k)
        end = names.index(b"\0", sh_name)
        if names[sh_name:end].decode() == name:
            if sh_type == 8:  # SHT_NOBITS
                return b""
            return data[off:off + size]
    raise KeyError(f"{path}: no section {name}")


def code_objects(path: str, arch: str = "gfx950") -> list[bytes]:
    """The `arch` code objects of every offload bundle in the file."""
    fatbin = elf_section(path, ".hip_fatbin")
    out = []
    pos = fatbin.find(BUNDLE_MAGIC)
    while pos >= 0:
        count, = struct.unpack_from("<Q", fatbin, pos + len(BUNDLE_MAGIC))
        cur = pos + len(BUNDLE_MAGIC) + 8
        for _ in range(count):
            off, size, tlen = struct.unpack_from("<QQQ", fatbin, cur)
            triple = fatbin[cur + 24:cur + 24 + tlen].decode()
            cur += 24 + tlen
            if "amdgcn" in triple and triple.endswith(arch) and size:
                blob = fatbin[pos + off:pos + off + size]
                if blob[:4] != b"\x7fELF":
                    raise ValueError(f"{path}: {triple} entry is not a plain ELF code object")
                out.append(blob)
        pos = fatbin.find(BUNDLE_MAGIC, cur)
    return out


def disassemble(blob: bytes, arch: str = "gfx950") -> list[str]:
    """Instruction lines (mnemonic and operands, no comments) of a code
    object, with each function's label line kept as '<name>:'."""
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "code.co")
        with open(f, "wb") as fh:
            fh.write(blob)
        r = subprocess.run([OBJDUMP, "-d", f"--mcpu={arch}", f], capture_output=True, text=True, check=True)
    lines = []
    for raw in r.stdout.splitlines():
        s = raw.split("//", 1)[0].strip()
        if not s:
            continue
        if s.endswith(">:"):
            lines.append(s)
        elif raw.startswith("\t") or raw.startswith(" "):
            lines.append(s)
    return lines


def vgprs(operand: str) -> set[int]:
    """Vector registers named in one operand (v7, v[8:11])."""
    regs = set()
    for m in re.finditer(r"\bv\[(\d+):(\d+)\]", operand):
        regs.update(range(int(m.group(1)), int(m.group(2)) + 1))
    for m in re.finditer(r"\bv(\d+)\b", operand):
        regs.add(int(m.group(1)))
    return regs


WIDE_STORE = re.compile(r"^(global|flat|buffer)_store_dwordx[34]\b")
BRANCH = re.compile(r"^s_(c?branch|setpc|swappc|endpgm|trap)")


def store_data_hazards(lines: list[str], wait_states: int = 2, only=None):
    """Wide (96- or 128-bit) vector stores whose data registers a VALU
    instruction overwrites fewer than `wait_states` wait states after the
    store.  Each instruction counts one wait state and s_nop N counts N + 1.
    The scan follows straight-line code only: a store whose window is still
    open at a branch, the end of the program or a function boundary is
    counted as unresolved.  `only` filters the stores checked (a predicate
    on the line).  Returns (stores checked, offending store lines with the
    instruction that broke the window, unresolved store lines)."""
    checked, bad, unresolved = 0, [], []
    n = len(lines)
    for i, line in enumerate(lines):
        if not WIDE_STORE.match(line) or (only and not only(line)):
            continue
        checked += 1
        ops = line.split(None, 1)[1].split(",")
        # data is the first operand of a buffer store, the second of a
        # global or flat store (after the address)
        data = vgprs(ops[0] if line.startswith("buffer_") else ops[1])
        waited = 0
        k = i + 1
        while waited < wait_states:
            if k >= n or lines[k].endswith(">:"):
                unresolved.append(line)
                break
            nxt = lines[k]
            k += 1
            if BRANCH.match(nxt):
                waited += 1
                if waited < wait_states:
                    unresolved.append(f"{line}  ->  {nxt}")
                break
            if nxt.startswith("s_nop"):
                waited += int(nxt.split()[1], 0) + 1
                continue
            if nxt.startswith("v_") and " " in nxt:
                if vgprs(nxt.split(None, 1)[1].split(",")[0]) & data:
                    bad.append(f"{line}  ->  {nxt}")
                    break
            waited += 1
    return checked, bad, unresolved
