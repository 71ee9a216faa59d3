"""CPU model of the reverse blend's DPP reduce-scatter (the `row_sums9` asm
block in csrc/blend.hip).  The test reads the instruction sequence from the
source, runs it on a model of one 16-lane DPP row and checks that the lanes
end with the row totals the kernel's LDS adds assume: bank b (lanes 4b..4b+3)
holds value {0,2,1,3}[b] in operand 0 and value 4 + {0,2,1,3}[b] in operand 4,
every lane holds value 8 in operand 8.  It also checks the DPP read hazard
inside the block: a DPP source is read at least two instructions after its
last write (the block opens with s_nop 1 for its inputs).

Model of the GFX9 DPP forms used: row_ror:n reads lane (l - n) mod 16 of the
row, quad_perm:[a,b,c,d] reads lane 4 (l / 4) + perm[l % 4], and a lane whose
bank bit is clear in bank_mask keeps its destination."""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2605_06876_amd", "csrc", "blend.hip")
INSN = re.compile(r'"v_add_f32_dpp %(\d), %(\d), %(\d) (row_ror:(\d+)|quad_perm:\[([0-3]),([0-3]),([0-3]),([0-3])\]) '
                  r'row_mask:0xf bank_mask:0x([0-9a-f])')


def _block():
    src = open(SRC).read()
    body = src[src.index("void row_sums9("):]
    body = body[:body.index(": \"+v\"(g[0])")]
    assert '"s_nop 1' in body
    seq = []
    for m in INSN.finditer(body):
        d, a, b = int(m.group(1)), int(m.group(2)), int(m.group(3))
        if m.group(5):
            ctrl = ("ror", int(m.group(5)))
        else:
            ctrl = ("quad", [int(m.group(k)) for k in range(6, 10)])
        seq.append((d, a, b, ctrl, int(m.group(10), 16)))
    return seq


def _run(seq, g):
    R = [g[k].copy() for k in range(9)]
    for d, a, b, ctrl, bm in seq:
        out = R[d].copy()
        for l in range(16):
            if not (bm >> (l // 4)) & 1:
                continue
            sl = (l - ctrl[1]) % 16 if ctrl[0] == "ror" else 4 * (l // 4) + ctrl[1][l % 4]
            out[l] = R[a][sl] + R[b][l]
        R[d] = out
    return R


def test_sequence_is_the_documented_reduce_scatter():
    seq = _block()
    assert len(seq) == 20
    rng = np.random.default_rng(7)
    for _ in range(20):
        g = rng.integers(-1000, 1000, size=(9, 16)).astype(np.float64)   # exact sums
        R = _run(seq, g)
        tot = g.sum(1)
        for l in range(16):
            b = l // 4
            k0 = ((b & 1) << 1) | (b >> 1)
            assert R[0][l] == tot[k0]
            assert R[4][l] == tot[4 + k0]
            assert R[8][l] == tot[8]


def test_a_planted_wrong_rotation_is_caught():
    seq = _block()
    bad = [(d, a, b, ("ror", 16 - c[1]) if c[0] == "ror" and c[1] in (4, 12) and m != 0xF else c, m)
           for d, a, b, c, m in seq]
    g = np.random.default_rng(1).integers(-9, 9, size=(9, 16)).astype(np.float64)
    R = _run(bad, g)
    assert not all(R[0][l] == g.sum(1)[((l // 4 & 1) << 1) | (l // 8)] for l in range(16))


def test_dpp_sources_are_read_two_instructions_after_their_last_write():
    seq = _block()
    last = {}
    for i, (d, a, b, _, _) in enumerate(seq):
        if a in last:
            assert i - last[a] >= 3, (i, a)   # two instructions in between
        last[d] = i
