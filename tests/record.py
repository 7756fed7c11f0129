"""Helpers of the full-size parity tests.

* record(): result lines, printed and appended as JSON to the file named by the environment variable
  DTB_ACCURACY_LOG (if set), with the hash of the kernel sources measured.
* oracle_in_chunks(): an oracle run of many steps as consecutive shorter runs (the result is the same bit
  for bit: running T1 steps and then T2 steps is running T1 + T2 steps, a pinned property of the oracle),
  printing progress between them so that a long run is never silent.
"""
import json
import os
import sys
import time

from paper_2306_03336_amd import build


def record(**kv):
    kv["kernel_source_sha256"] = build.kernel_source_hash()
    print("[result]", json.dumps(kv), flush=True)
    path = os.environ.get("DTB_ACCURACY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(kv) + "\n")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_in_chunks(fn, u, coeffs, T, label, chunk=200):
    t0 = time.perf_counter()
    done = 0
    while done < T:
        n = min(chunk, T - done)
        u = fn(u, coeffs, n)
        done += n
        say(f"[oracle] {label}: {done}/{T} steps, {time.perf_counter() - t0:.0f} s")
    return u
