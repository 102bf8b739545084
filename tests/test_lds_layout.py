"""The swizzled LDS layout of the 512-, 1024- and 2048-point transforms
(dh_fft.hpp), checked on the CPU from the header itself (a host-only build of
tests/lds_layout_dump.cpp):

- the slot map is a bijection of [0, N) that changes the low four bits only
  and is linear over XOR, which is what lets every pass split an address into
  a per-lane part and a compile-time offset;
- under the gfx950 LDS bank model (64-bit reads: 32 lanes per cycle over 32
  banks of 8 bytes; 64-bit writes: 16 lanes per cycle, bank = slot mod 16),
  every read and write of the Stockham passes is free of bank conflicts, where
  the padded layout (i + i / R0) is not (a check that the model sees them).
"""
import os
import shutil
import subprocess
import tempfile
from collections import defaultdict

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2204_02348_amd", "csrc")


@pytest.fixture(scope="module")
def layouts():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "lds_layout_dump")
        subprocess.run([hipcc, "-std=c++17", "-x", "hip", "--offload-host-only", "-I", CSRC,
                        os.path.join(HERE, "lds_layout_dump.cpp"), "-o", exe],
                       check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    res = {}
    for k in range(0, len(out) - 1, 2):
        h = out[k].split()
        n = int(h[1])
        res[n] = dict(swz=bool(int(h[3])), stride=int(h[5]), radices=[int(x) for x in h[7:10] if int(x) > 1],
                      slot=[int(x) for x in out[k + 1].split()])
    return res


def _conflicts(addrs, lanes_per_cycle, banks):
    """extra cycles of one 64-lane instruction (None: inactive lane)"""
    extra = 0
    for h in range(0, 64, lanes_per_cycle):
        per = defaultdict(set)
        for a in addrs[h:h + lanes_per_cycle]:
            if a is not None:
                per[a % banks].add(a)
        extra += max((len(v) for v in per.values()), default=1) - 1
    return extra


def _pass_conflicts(n, radices, at, ntr=8, tpb=256):
    """(read, write) conflict cycles of every Stockham pass of ntr transforms
    of n points at stride n + 4 (butterfly g = tid + it tpb: transform g / NB,
    butterfly g % NB; pass 1 writes R0-element blocks, later passes read the
    R elements NB apart and write them NS apart)"""
    st = n + 4
    rd = wr = 0
    ns = 1
    for s, r in enumerate(radices):
        nb = n // r
        total = ntr * nb
        for w in range(tpb // 64):
            for it in range((total + tpb - 1) // tpb):
                g = [w * 64 + l + it * tpb for l in range(64)]
                ok = [x < total for x in g]
                if s > 0:
                    for q in range(r):
                        rd += _conflicts([(x // nb) * st + at(x % nb + q * nb) if o else None
                                          for x, o in zip(g, ok)], 32, 32)
                for q in range(r):
                    if s == 0:
                        ad = [(x // nb) * st + at((x % nb) * r + q) if o else None for x, o in zip(g, ok)]
                    else:
                        ad = [(x // nb) * st + at((x % nb) // ns * ns * r + (x % nb) % ns + q * ns) if o else None
                              for x, o in zip(g, ok)]
                    wr += _conflicts(ad, 16, 16)
        ns *= r
    return rd, wr


@pytest.mark.parametrize("n", [512, 1024, 2048])
def test_swizzle_is_a_linear_bijection_of_the_low_bits(layouts, n):
    L = layouts[n]
    assert L["swz"] and L["stride"] == n + 4
    slot = L["slot"]
    assert sorted(slot) == list(range(n))
    assert all((s ^ i) & ~15 == 0 for i, s in enumerate(slot))
    for x in range(n):                               # linear over XOR: the slot of x is
        acc = 0                                      # the XOR of the slots of its bits
        for b in range(n.bit_length()):
            if x >> b & 1:
                acc ^= slot[1 << b]
        assert slot[x] == acc, x


@pytest.mark.parametrize("n", [512, 1024, 2048])
def test_swizzled_passes_are_free_of_bank_conflicts(layouts, n):
    L = layouts[n]
    rd, wr = _pass_conflicts(n, L["radices"], lambda i: L["slot"][i])
    assert (rd, wr) == (0, 0)
    r0 = L["radices"][0]
    prd, pwr = _pass_conflicts(n, L["radices"], lambda i: i + i // r0)
    assert prd + pwr > 0                              # the model does see the padded layout's
