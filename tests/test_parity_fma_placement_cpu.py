"""Placement of the parity step in the generated gfx950 code (host only: the
kernels are compiled to device assembly, nothing runs on a GPU).

On the grid schedule the FP32 sweep kernels switch the wave's FP32 rounding
mode to round-toward-minus-infinity and take Eq. (4)'s sign from an fma whose
addend is 1.5 * 2^23.  The compiler does not order instructions against a
write of the MODE register, so the switch yields that addend and every parity
fma must take it from there.  Checked here, for every kernel instantiation
that switches the mode: it has parity fmas, each reads the scalar register the
switch wrote, each lies after a round-down switch with no switch back in
between, and no fma adds the constant as a literal (which the compiler could
schedule before the switch)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_30355_amd", "csrc")
SOURCES = ["sweep_stream.hip", "kernels.hip", "sweep_reg.hip", "sweep_rstream.hip", "batch.hip"]
FLAGS = ["-O3", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
         "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "--cuda-device-only", "-S", "-x", "hip"]


def functions(asm):
    out, cur = [], None
    for line in asm.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            cur = (m.group(1), [])
            out.append(cur)
        elif cur is not None:
            cur[1].append(line.strip())
    return out


def compile_all(tmp_path):
    """Device assembly of every source, compiled side by side."""
    procs = {}
    for src in SOURCES:
        out = str(tmp_path / (src + ".s"))
        procs[src] = (out, subprocess.Popen(["hipcc", *FLAGS, os.path.join(CSRC, src), "-o", out],
                                            stdout=subprocess.PIPE, stderr=subprocess.PIPE))
    result = {}
    for src, (out, p) in procs.items():
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, err.decode()[-2000:]
        with open(out) as f:
            result[src] = f.read()
    return result


def test_parity_fmas_inside_the_round_down_window(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    down_re = re.compile(r"s_setreg_imm32_b32 hwreg\(HW_REG_MODE, 0, 2\), 2")
    up_re = re.compile(r"s_setreg_imm32_b32 hwreg\(HW_REG_MODE, 0, 2\), 0")
    magic_re = re.compile(r"s_mov_b32 (s\d+), 0x4b400000")
    for src, asm in compile_all(tmp_path).items():
        switching = 0
        for name, body in functions(asm):
            if not any(down_re.search(l) for l in body):
                assert not any(up_re.search(l) for l in body), name
                continue
            switching += 1
            assert not any(l.startswith(("v_fmaak_f32", "v_fmamk_f32")) and "0x4b400000" in l
                           for l in body), f"{name}: the addend as a literal"
            state, sreg, n_fma = None, None, 0
            for line in body:
                if down_re.search(line):
                    state = "down"
                elif up_re.search(line):
                    state = "nearest"
                m = magic_re.search(line)
                if m:
                    sreg = m.group(1)
                if sreg and line.startswith("v_fma_f32") and line.endswith(", " + sreg):
                    n_fma += 1
                    assert state == "down", f"{name}: {line} outside the round-down window"
            assert n_fma > 0, f"{name}: switches the mode but has no parity fma"
        assert switching > 0, f"{src}: no kernel switches the rounding mode"
