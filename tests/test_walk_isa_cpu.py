"""The persistent walk's queue claims, checked in the gfx950 code the build
makes of k_walk.hip (CPU only: hipcc compiles, nothing runs).

Every wavefront of the walk loops claiming queue positions until the queue
is empty. The loop must contain no region that only some lanes enter and that
the compiler can thread across the loop's back edge: a wavefront that
re-enters the loop with part of its lanes masked off reads a stale queue
position and never leaves. The source therefore has every lane join each
claim (lane 0 adds 1, the others 0) and takes the position through
readfirstlane. In the machine code that shows as: each returning atomic add
of the walk kernels sits alone in a one-lane region (the compiler's own
single-lane election for a wave-wide atomic), the region closes right after
it, and the result is made wave-uniform by v_readfirstlane_b32 at once."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_1811_02761_amd"))
import build  # noqa: E402

WALK_KERNELS = ("k_walk", "k_walk_retry", "k_walk_pot")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("walk_isa") / "k_walk.s")
    flags = [f for f in build.FLAGS if f != "-fPIC"]
    cmd = [build.HIPCC, *flags, "--cuda-device-only", "-S",
           os.path.join(build.CSRC, "k_walk.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    with open(out) as f:
        return f.read()


def functions(text):
    """{mangled name: list of instruction lines} of the walk kernels."""
    funcs = {}
    pat = re.compile(r"^(_ZN2nb(\d+)(k_walk\w*?)I\w*):", re.M)
    for m in pat.finditer(text):
        name, ln, base = m.group(1), int(m.group(2)), m.group(3)
        if base[:ln] not in WALK_KERNELS:
            continue
        body = text[m.end():text.index("s_endpgm", m.end())]
        lines = [l.split(";")[0].strip() for l in body.splitlines()]
        funcs[name] = [l for l in lines if l]
    return funcs


def test_every_walk_kernel_is_checked(asm):
    names = functions(asm)
    # the main pass, the retry pass and the potential variant, each in the
    # plain / compensated and hash / no-hash forms
    for k in WALK_KERNELS:
        tag = "%d%s" % (len(k), k)
        assert sum(tag + "I" in n for n in names) == 4, (k, sorted(names))


def test_queue_claims_are_wave_uniform(asm):
    for name, ins in functions(asm).items():
        claims = [i for i, l in enumerate(ins)
                  if l.startswith("global_atomic_add ") and re.search(r"\bsc0\b", l)]
        assert claims, "%s: no returning atomic add (the queue claim)" % name
        for i in claims:
            # the one-lane region around the atomic: opened by saveexec just
            # before it (only the election's mask bookkeeping between) ...
            j = i - 1
            while j >= 0 and not ins[j].startswith("s_and_saveexec_b64"):
                assert ins[j].endswith(":") or re.match(
                    r"(s_xor_b64 s\[\d+:\d+\], exec|s_cbranch_execz|v_mov_b32)", ins[j]), \
                    "%s: %r inside the claim's lane mask" % (name, ins[j])
                j -= 1
            assert j >= 0 and i - j <= 6, "%s: claim region not found" % name
            # ... closed right after it, then the result made wave-uniform
            k = i + 1
            while ins[k].endswith(":"):
                k += 1
            assert ins[k].startswith("s_or_b64 exec, exec,"), \
                "%s: %r after the claim" % (name, ins[k])
            nxt = ins[k + 1:k + 4]
            assert any(l.startswith("v_readfirstlane_b32") for l in nxt), \
                "%s: claim result not made uniform: %r" % (name, nxt)
