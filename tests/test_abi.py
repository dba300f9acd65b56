"""The C-ABI library loads, exports every function include/pmp.h declares, and
the Python binding's structures have the C layout (checked against a small C
program compiled from the header).  No GPU needed."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2509_18261_amd import binding as B
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(B.lib, n), n
    bound = {s[0] for s in B.SIGNATURES}
    assert bound == set(names), (bound ^ set(names))


def test_nm_exports():
    lib = os.path.join(ROOT, "paper_2509_18261_amd", "libpmp.so")
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pmp_[a-z_]+)\b", out))
    assert set(declared_functions()) <= exported


STRUCTS = {
    "pmp_layout": ["nbox", "lo", "n", "ghost", "domain", "dx", "acc", "state", "with_sinks",
                   "channels"],
    "pmp_cic": ["x", "y", "z", "m", "n", "box_off"],
    "pmp_sn": ["x", "y", "z", "m", "e", "r", "n", "box_off", "r_max"],
    "pmp_sinks": ["x", "y", "z", "a", "n", "box_off", "r_k", "r_gauss", "rate", "m", "vx",
                  "vy", "vz", "G", "dt", "gamma", "lambda"],
    "pmp_snr": ["x", "y", "z", "m", "e", "vx", "vy", "vz", "n", "box_off", "r_k", "sub",
                "nh_per_rho", "msf_coef", "psnr_coef", "eps_k"],
    "pmp_limits": ["rho_floor", "rho_tr", "cap", "eint_mode", "truelove_J", "G", "gamma"],
    "pmp_status": ["flags", "reserved", "touched", "bind", "lam", "fall"],
    "pmp_tuning": ["deposit_path", "tile_x", "tile_yz", "tile_block", "block", "grid_per_cu",
                   "sn_lanes", "tile_grid_per_cu", "chunk_cic", "chunk_sn",
                   "fuse_apply", "count_lanes"],
}


def test_struct_layout_matches_header(tmp_path):
    from paper_2509_18261_amd import binding as B
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"',
             "int main(void) {"]
    for s, fields in STRUCTS.items():
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for f in fields:
            lines.append(f'printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    for line in out.strip().splitlines():
        s, f, v = line.split()
        cls = getattr(B, s)
        if f == "size":
            assert C_sizeof(cls) == int(v), line
        else:
            # "lambda" is a Python keyword: the binding names that field "lambda_"
            assert getattr(cls, "lambda_" if f == "lambda" else f).offset == int(v), line


def C_sizeof(cls):
    import ctypes
    return ctypes.sizeof(cls)


def test_no_cpu_fallback_in_binding():
    """The binding refuses to run without the HIP library."""
    text = open(os.path.join(ROOT, "paper_2509_18261_amd", "binding.py")).read()
    assert "oracle" not in text
    assert "raise ImportError" in text
