"""Structure of the compiled queue loops (CPU only: compiles the library to gfx950 assembly).

Every mid/heavy/batched kernel pulls work items with one atomic on a device
counter, done by thread 0, followed by two workgroup barriers that publish
the item to all threads. The item's work must end convergent. If a lane-0-
only store ends an item with no barrier after it, the compiler can turn the
queue loop into a nested loop whose back edge skips the atomic for every
lane but thread 0's. Those lanes then re-read the old item forever (a GPU
hang). This test checks the assembly: no loop header lies between the
atomic and its two barriers (the atomic sits in the queue loop, which is
the outermost loop or, for the per-XCD queues, the loop inside the one over
the XCDs' queues).

A second check: no kernel calls a device function. The kernels take the plan
descriptor by value and the tier functions take it by reference; a call that
is not inlined makes the compiler copy the whole descriptor into per-lane
scratch memory at kernel entry and read every field from there, which
slowed the single persistent launch by about a quarter when the output-mask
code pushed the tier functions past the inliner's size limit.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1006_2183_amd", "csrc", "sg_spgemm.hip")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    return _asm(str(tmp_path_factory.mktemp("asm")))


def _asm(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = os.path.join(tmp_path, "sg.s")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                           "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics", "-I" + os.path.join(ROOT, "include"),
                           "--cuda-device-only", "-S", "-o", out, SRC],
                          stderr=subprocess.DEVNULL)
    with open(out) as f:
        return f.read()


def queue_loop_report(asm: str):
    rows = []
    for m in re.finditer(r"^(_ZN2sg(?:5k_mid|7k_heavy|9k_batched|11k_mid_count|13k_heavy_count)\S*):.*?s_endpgm", asm, re.S | re.M):
        name, body = m.group(1), m.group(0)
        lines = body.split("\n")
        atom = [i for i, l in enumerate(lines) if "global_atomic_add_x2" in l]
        if not atom:
            rows.append((name, False, "no queue atomic"))
            continue
        a = atom[0]
        headers = [l for l in lines[:a] if "Loop Header: Depth=" in l]
        depth = re.search(r"Depth=(\d+)", headers[-1]).group(1) if headers else None
        bars = [i for i in range(a, len(lines)) if "s_barrier" in lines[i]][:2]
        between = [l for l in lines[a:bars[-1]] if "Loop Header" in l] if len(bars) == 2 else ["?"]
        ok = depth in ("1", "2") and len(bars) == 2 and not between
        rows.append((name, ok, f"atomic at loop depth {depth}, loop headers before its barriers: {len(between)}"))
    return rows


def test_queue_loops_stay_convergent(asm):
    rows = queue_loop_report(asm)
    # 4 semirings x (mid count and numeric, heavy count per window kind, heavy numeric per window kind
    # plus rank windows with entry records, batched per kind set plus the two with rank windows and records)
    assert len(rows) == 48, f"expected 48 queue kernels, found {len(rows)}"
    bad = [r for r in rows if not r[1]]
    assert not bad, "queue loop restructured: " + "; ".join(f"{n}: {why}" for n, _, why in bad)


def calls_report(asm: str):
    """(kernel, called symbols) for every kernel whose body makes a call."""
    rows = []
    for m in re.finditer(r"^(_ZN2sg\d+k_\S*):.*?s_endpgm", asm, re.S | re.M):
        body = m.group(0)
        if "s_swappc_b64" in body:
            rows.append((m.group(1), sorted(set(re.findall(r"(_Z\w+)@rel32@lo", body)))))
    return rows


def test_kernels_make_no_calls(asm):
    bad = calls_report(asm)
    assert not bad, "kernels calling device functions: " + "; ".join(f"{k} -> {c}" for k, c in bad)
