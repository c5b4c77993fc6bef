"""The AMD assembly of the library's kernels (built here for gfx950, no GPU needed): the
FP32 Euler step must not contain fused multiply-adds, since the oracle rounds every
product and sum on its own (the build passes -ffp-contract=off; this checks the result),
and no kernel may use packed FP32 arithmetic (the build disables it)."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

FUSED = re.compile(r"\b(v_fma_f32|v_fmac_f32|v_fmamk_f32|v_fmaak_f32|v_mad_f32|v_mac_f32|v_madmk_f32|v_madak_f32|"
                   r"v_fma_mix\w*|v_mad_mix\w*|v_fma_f64|v_fmac_f64|v_pk_fma_f32)\b")
PACKED = re.compile(r"\b(v_pk_add_f32|v_pk_mul_f32|v_pk_fma_f32)\b")
FP32_FUSED = re.compile(r"\b(v_fma_f32|v_fmac_f32|v_fmamk_f32|v_fmaak_f32|v_mad_f32|v_mac_f32|v_fma_mix\w*|"
                        r"v_mad_mix\w*)\b")


@pytest.fixture(scope="module")
def asm():
    from paper_2211_15963_amd import build as b
    out = os.path.join(tempfile.mkdtemp(), "kernels.s")
    src = os.path.join(ROOT, "paper_2211_15963_amd", "csrc", "kernels.hip")
    subprocess.run([b.hipcc(), "-x", "hip", *b.HIPFLAGS, "--cuda-device-only", "-S", src, "-o", out], check=True,
                   capture_output=True)
    funcs, cur = {}, None
    for line in open(out):
        m = re.match(r"^(_Z\w+):", line)
        if m:
            cur = m.group(1)
            funcs[cur] = []
        elif cur is not None:
            funcs[cur].append(line)
            if "s_endpgm" in line:
                cur = None
    return funcs


def _named(funcs, part):
    got = {k: v for k, v in funcs.items() if part in k}
    assert got, f"no kernel named like {part}"
    return got


def test_euler_step_has_no_fused_operations(asm):
    for name, body in _named(asm, "k_neuron").items():
        text = "".join(body)
        assert "v_mul_f32" in text and "v_add_f32" in text, name
        bad = sorted(set(FUSED.findall(text)))
        assert not bad, f"{name}: {bad}"


def test_gather_conversion_has_no_fused_fp32(asm):
    for name, body in _named(asm, "k_gather").items():
        bad = sorted(set(FP32_FUSED.findall("".join(body))))
        assert not bad, f"{name}: {bad}"


def test_no_packed_fp32_anywhere(asm):
    for name, body in asm.items():
        bad = sorted(set(PACKED.findall("".join(body))))
        assert not bad, f"{name}: {bad}"
