"""C-ABI checks that need no GPU: the library loads, it exports every function
include/mpm.h declares, and the ctypes structs of the Python binding have the
layout the C compiler gives the header's structs."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s*(mpm_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ("mpm_create", "mpm_set_particles", "mpm_set_tool_sdf", "mpm_step", "mpm_read_state"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2502_18437_amd import mpm
    names = declared_functions()
    missing = [n for n in names if not hasattr(mpm._lib, n)]
    assert not missing, missing
    assert set(names) == set(mpm.EXPORTED)
    nm = subprocess.run(["nm", "-D", "--defined-only", mpm.LIB_PATH], capture_output=True, text=True)
    exported = set(re.findall(r" T (mpm_\w+)$", nm.stdout, flags=re.M))
    assert set(names) <= exported


LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "mpm.h"
#define F(T, m) printf(#T " " #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("mpm_params SIZEOF %zu\n", sizeof(mpm_params));
  F(mpm_params, n_grid) F(mpm_params, dt) F(mpm_params, gravity) F(mpm_params, wall_band)
  F(mpm_params, nu) F(mpm_params, E_default) F(mpm_params, accum_mode) F(mpm_params, tile)
  F(mpm_params, resort_interval) F(mpm_params, max_particles)
  printf("mpm_tool SIZEOF %zu\n", sizeof(mpm_tool));
  F(mpm_tool, type) F(mpm_tool, center) F(mpm_tool, quat) F(mpm_tool, size) F(mpm_tool, lin_vel)
  F(mpm_tool, ang_vel) F(mpm_tool, mu) F(mpm_tool, drag) F(mpm_tool, margin) F(mpm_tool, push_out)
  printf("mpm_info SIZEOF %zu\n", sizeof(mpm_info));
  F(mpm_info, n_particles) F(mpm_info, n_fallback) F(mpm_info, n_range) F(mpm_info, tile) F(mpm_info, n_tools) F(mpm_info, rollouts)
  printf("mpm_launch_config SIZEOF %zu\n", sizeof(mpm_launch_config));
  F(mpm_launch_config, resort_interval) F(mpm_launch_config, transfer_wgs) F(mpm_launch_config, graph_chunk) F(mpm_launch_config, rebin_mode) F(mpm_launch_config, tile) F(mpm_launch_config, rebin_drift)
  printf("mpm_kernel_times SIZEOF %zu\n", sizeof(mpm_kernel_times));
  F(mpm_kernel_times, total_ms) F(mpm_kernel_times, launches)
  return 0;
}
"""


def test_struct_layouts_match_ctypes(tmp_path):
    from paper_2502_18437_amd import mpm
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    structs = {"mpm_params": mpm.mpm_params, "mpm_tool": mpm.mpm_tool, "mpm_info": mpm.mpm_info,
               "mpm_kernel_times": mpm.mpm_kernel_times, "mpm_launch_config": mpm.mpm_launch_config}
    for line in out:
        if not line:
            continue
        sname, field, val = line.split()
        cls = structs[sname]
        if field == "SIZEOF":
            assert mpm.ctypes.sizeof(cls) == int(val), sname
        else:
            assert getattr(cls, field).offset == int(val), (sname, field)


def test_status_codes_match_header():
    from paper_2502_18437_amd import mpm
    text = open(HEADER).read()
    for name in ("MPM_OK", "MPM_EINVAL", "MPM_ENOMEM", "MPM_EHIP", "MPM_EDOMAIN", "MPM_ENONFINITE",
                 "MPM_EINVERTED", "MPM_ERANGE", "MPM_HOST", "MPM_DEVICE", "MPM_TOOL_CAPSULE", "MPM_TOOL_BOX",
                 "MPM_TOOL_PLANE", "MPM_ACCUM_FIXED", "MPM_KERNEL_KINDS", "MPM_MAX_TOOLS", "MPM_SOLVER_MLS",
                 "MPM_SOLVER_PIC", "MPM_SOLVER_PB", "MPM_REBIN_AUTO", "MPM_REBIN_ADVANCE", "MPM_REBIN_IN_PLACE"):
        m = re.search(r"#define\s+%s\s+\(?(-?\d+)\)?" % name, text)
        assert m, name
        assert getattr(mpm, name) == int(m.group(1)), name


def test_null_handle_calls_are_rejected_without_a_gpu():
    """Argument validation happens before any device work."""
    from paper_2502_18437_amd import mpm
    assert mpm._lib.mpm_step(None, 1) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_destroy(None) == mpm.MPM_OK
    assert mpm._lib.mpm_set_tool_sdf(None, 0, None) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_create(None, 0, None) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_eval_stress(-1, None, None, 0.3, None, 0) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_set_tool_velocity_table(None, 0, 0, None) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_rollout_forward(None, 1, 1, None) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_rollout_backward(None, *([None] * 10)) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_set_launch_config(None, None) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_autotune(None, 1, None) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_set_solver(None, mpm.MPM_SOLVER_PB, 10, 0.5) == mpm.MPM_EINVAL
    assert mpm._lib.mpm_get_solver(None, None, None, None) == mpm.MPM_EINVAL


def _device_kernel_descriptors(path):
    """(name, group_segment, private_segment, kernel_code_properties) of every
    kernel in the gfx950 code objects that the built library bundles
    (clang offload bundles, uncompressed, one per source file)."""
    import struct
    data = open(path, "rb").read()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    out = []
    pos = data.find(magic)
    while pos >= 0:
        (n_entries,) = struct.unpack_from("<Q", data, pos + 24)
        q = pos + 32
        for _ in range(n_entries):
            off, size, tlen = struct.unpack_from("<QQQ", data, q)
            triple = data[q + 24:q + 24 + tlen].decode()
            q += 24 + tlen
            if "gfx950" not in triple:
                continue
            elf = data[pos + off:pos + off + size]
            assert elf[:4] == b"\x7fELF"
            shoff, = struct.unpack_from("<Q", elf, 0x28)
            shentsize, shnum = struct.unpack_from("<HH", elf, 0x3A)
            secs = [struct.unpack_from("<IIQQQQIIQQ", elf, shoff + i * shentsize) for i in range(shnum)]
            symtab = next(sh for sh in secs if sh[1] == 2)  # SHT_SYMTAB
            strtab = secs[symtab[6]]
            for k in range(symtab[5] // 24):
                st_name, st_info, st_other, st_shndx, st_value, st_size = struct.unpack_from(
                    "<IBBHQQ", elf, symtab[4] + 24 * k)
                end = elf.index(b"\0", strtab[4] + st_name)
                name = elf[strtab[4] + st_name:end].decode()
                if not name.endswith(".kd"):
                    continue
                sec = secs[st_shndx]
                kd = sec[4] + (st_value - sec[3])
                group, private = struct.unpack_from("<II", elf, kd)
                (props,) = struct.unpack_from("<H", elf, kd + 56)
                out.append((name[:-3], group, private, props))
        pos = data.find(magic, pos + 1)
    return out


def test_kernels_use_no_scratch_and_do_not_read_the_dispatch_packet():
    """Every device kernel runs without scratch memory and without the
    dispatch pointer. A per-thread array indexed at run time makes the
    compiler keep it in scratch or in LDS at an offset of the flat work-item
    id, whose computation reads the workgroup size from the dispatch packet
    in every wave; that once cost a 5.5 us kernel 13 us."""
    from paper_2502_18437_amd import mpm
    kds = _device_kernel_descriptors(mpm.LIB_PATH)
    names = [k[0] for k in kds]
    assert any("k_g2p2g" in n for n in names) and any("k_bgrid" in n for n in names), names[:5]
    for name, group, private, props in kds:
        assert private == 0, (name, private)
        assert not props & 0x2, name  # ENABLE_SGPR_DISPATCH_PTR
