"""The batched solve's host plan under AddressSanitizer and UBSan (CPU only).

The host driver is built with both sanitizers (the kernel objects as usual)
and loaded into a child process that preloads the sanitizer runtime.  In it,
slse_debug_batch_plan builds and bounds-checks the whole plan (pools and
offsets, SRHT job and record tables, factor jobs, per-step tile tables) for
the batched workload's 64 problems, for its 6-problem sample and for a batch
of mixed sketch kinds; any heap or stack overflow, use after free or
undefined behaviour in that host code ends the child with a report.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import torch
    from oracle import slse as OS
    from paper_2509_06856_amd import slse as G
    from slse_inputs import batched_shapes

    def params(shapes, kinds, factor="chol"):
        out = []
        for i, (n, d) in enumerate(shapes):
            m = OS.paper_schedule(n, d)
            out.append(G.Params(kind=kinds[i % len(kinds)], seed=2000 + i, m=m, a=[2] * len(m),
                                r=6 * d, s_max=45, precision="mixed", factor=factor))
        return out

    for shapes in (batched_shapes(count=6, n_range=(1 << 14, 1 << 15)), batched_shapes()):
        print("plan", len(shapes), G.debug_batch_plan(shapes, params(shapes, ["srht"])), flush=True)
    mixed = [(900, 8), (3000, 12), (6000, 16), (11000, 8), (2500, 10), (1800, 6), (40000, 40)]
    print("plan kinds", G.debug_batch_plan(mixed, params(mixed, ["srht", "countsketch", "gaussian"])))
    print("plan qr", G.debug_batch_plan(mixed, params(mixed, ["srht", "countsketch"], "qr")))
    print("schedule", G.paper_schedule(1 << 20, 64), G.auto_a([512, 1024, 2048], 64))
    print("DONE", flush=True)
""")


def test_batch_plan_clean_under_asan_and_ubsan():
    from paper_2509_06856_amd import build as B

    try:
        runtime = B.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    if not B.asan_build_is_current():
        B.build_host_asan(verbose=False)
    env = dict(os.environ)
    env.update(LD_PRELOAD=runtime, SLSE_LIB=B.ASAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "DONE" in r.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
