"""Audit of the generated gfx950 code against the numerics the library
claims (no GPU needed: hipcc cross-compiles every source to assembly with
the library's own flags).

* every kernel descriptor keeps binary32 denormals (input and output) and
  round-to-nearest-even;
* no packed binary32 instruction appears anywhere;
* contraction is off: the Mul22 kernels hold exactly one fused multiply-add
  per element (the explicit TwoProd), and binary32 Horner none -- both gain
  fused instructions when built with contraction on.
"""
import glob
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_cs_0603115_amd import build as B

pytestmark = pytest.mark.slow

SOURCES = sorted(glob.glob(os.path.join(B.CSRC, "*.hip")))


@pytest.fixture(scope="module")
def assembly(tmp_path_factory):
    out = tmp_path_factory.mktemp("asm")

    def compile_one(src):
        dst = os.path.join(out, os.path.basename(src) + ".s")
        cmd = [B.hipcc(), *B.HIPCC_FLAGS, "--cuda-device-only", "-S", src, "-o", dst]
        proc = subprocess.run(cmd, capture_output=True, text=True)
        assert proc.returncode == 0, proc.stderr[-2000:]
        with open(dst) as f:
            return os.path.basename(src), f.read()

    with ThreadPoolExecutor(min(8, len(SOURCES))) as pool:
        return dict(pool.map(compile_one, SOURCES))


def _kernel_bodies(text):
    """{mangled kernel name: its instructions} from an assembly listing."""
    bodies = {}
    for m in re.finditer(r"^(_Z[^\s:]+):[^\n]*\n(.*?)^\.Lfunc_end\d+:", text, re.M | re.S):
        bodies[m.group(1)] = m.group(2)
    return bodies


def test_every_kernel_preserves_denormals_and_rounds_to_nearest(assembly):
    n = 0
    for name, text in assembly.items():
        kernels = len(re.findall(r"^\s*\.amdhsa_kernel\s", text, re.M))
        denorm = re.findall(r"\.amdhsa_float_denorm_mode_32\s+(\d+)", text)
        rounding = re.findall(r"\.amdhsa_float_round_mode_32\s+(\d+)", text)
        assert len(denorm) == kernels and len(rounding) == kernels, name
        assert set(denorm) <= {"3"} and set(rounding) <= {"0"}, (name, set(denorm), set(rounding))
        n += kernels
    assert n >= 20                                   # every kernel was seen


def test_no_packed_binary32_instructions(assembly):
    for name, text in assembly.items():
        found = re.findall(r"^\s+(v_pk_(?:fma|mul|add)_f32)\b", text, re.M)
        assert not found, (name, sorted(set(found)))


def test_contraction_is_off(assembly):
    # Built with contraction on, both kernels below gain fused instructions
    # (Mul22: (ah * bl) + (al * bh) fuses; binary32 Horner: (s * x) + c).
    fused = re.compile(r"^\s+(v_fma\w*|v_fmac\w*|v_mad\w*|v_mac\w*|v_pk_fma\w*)\b", re.M)
    ew = _kernel_bodies(assembly["ff_elementwise.hip"])
    # Mul22 with FMA TwoProd: exactly one v_fma_f32 per element, the TwoProd
    # error term (four elements per lane in the float4 form, two in the
    # lane-contiguous form)
    for pattern, per_lane in ((r"ew_vecINS_5Mul22E", 4), (r"ew_streamINS_5Mul22E", 2)):
        names = [k for k in ew if re.search(pattern, k)]
        assert len(names) == 1, (pattern, sorted(ew))
        assert fused.findall(ew[names[0]]) == ["v_fma_f32"] * per_lane, names[0]
    # Horner's rule in binary32: a multiply and an add per step, never fused
    poly = _kernel_bodies(assembly["ff_poly.hip"])
    horner = [k for k in poly if "HornerF32" in k]
    assert len(horner) == 8, sorted(poly)
    for k in horner:
        assert not fused.findall(poly[k]), k
