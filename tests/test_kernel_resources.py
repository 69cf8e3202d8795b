"""Register budget of the encoder+head kernels the benchmark times (CPU only: hipcc cross-compiles gfx950).

The BF16 encoder+head kernel of the split schedule and both FP8 kernels must keep every value in registers:
a spill writes scratch memory on every launch (8-10 MB per launch when it happened), traffic that the
kernels' HBM counter summaries would show and the roofline does not pay for.  The check reads the
resource metadata the compiler emits for each kernel (.vgpr_spill_count) at the scale widths
(128 / 256 / 512).
"""

import os
import subprocess

import pytest

from paper_2304_09439_amd import build as B

CSRC = os.path.join(B.PKG, "csrc")
INCLUDE = os.path.join(B.ROOT, "include")

# source file -> (demangled-name fragments of the kernels that must not spill)
KERNELS = {
    "fused.hip": ["fused_bf16_kernelILi128ELi256ELi512ELb1ELb0E",     # split schedule, contacts
                  "fused_bf16_kernelILi128ELi256ELi512ELb1ELb1E"],    # split schedule, argmax encoder
    "fused_fp8.hip": ["encoder_head_fp8_kernelILi128ELi256ELi512ELb1E",   # e4m3 encoder layer 2 and head
                      "encoder_head_fp8_kernelILi128ELi256ELi512ELb0E"],  # e4m3 encoder layer 2, bf16 head
}


def _spills(src, tmp_path):
    """{kernel symbol: (vgpr_count, vgpr_spill_count)} from the compiler's kernel metadata."""
    out = str(tmp_path / (src + ".s"))
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [B.hipcc(), *flags, "-I", INCLUDE, "-I", CSRC, "--cuda-device-only", "-S", "-o", out,
           os.path.join(CSRC, src)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    found, name, vgpr = {}, None, None
    for line in open(out):
        s = line.strip()
        if s.startswith(".name:"):
            name, vgpr = s.split(":", 1)[1].strip(), None
        elif s.startswith(".vgpr_count:") and name:
            vgpr = int(s.split(":", 1)[1])
        elif s.startswith(".vgpr_spill_count:") and name:
            found[name] = (vgpr, int(s.split(":", 1)[1]))
    return found


@pytest.mark.parametrize("src", sorted(KERNELS))
def test_encoder_head_kernels_do_not_spill(src, tmp_path):
    found = _spills(src, tmp_path)
    for frag in KERNELS[src]:
        hits = {k: v for k, v in found.items() if frag in k}
        assert hits, f"{frag} not in the metadata of {src}: {sorted(found)}"
        for k, (vgpr, spill) in hits.items():
            print(f"{k}: {vgpr} VGPRs, {spill} spilled")
            assert spill == 0, f"{k} spills {spill} VGPRs ({vgpr} VGPRs)"
