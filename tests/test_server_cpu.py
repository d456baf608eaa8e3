"""CPU checks of the quote server's host logic: the arena allocator that
admits quotes by memory (first fit in address order, coalescing on release,
never handing out overlapping ranges), driven against a Python model; and the
scheduler core with a stand-in executor backed by the oracle, under
ThreadSanitizer."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("arena") / "arena_driver")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_1308_2572_amd", "csrc"),
                           os.path.join(ROOT, "tests", "arena_driver.cpp"), "-o", exe])
    return exe


def run(exe, total, ops):
    out = subprocess.run([exe, str(total)], input="\n".join(ops) + "\n", capture_output=True, text=True, check=True)
    return out.stdout.split("\n")


class Model:
    def __init__(self, total):
        self.free = [(0, total)]

    def alloc(self, n):
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                if s == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, s - n)
                return o
        return None

    def release(self, o, n):
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for a, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((a, s))
        self.free = merged


@pytest.mark.parametrize("seed", range(6))
def test_arena_against_model(driver, seed):
    g = np.random.default_rng(seed)
    total = 10_000
    model = Model(total)
    live = []
    ops, expect = [], []
    for _ in range(400):
        if live and g.random() < 0.45:
            o, n = live.pop(int(g.integers(len(live))))
            ops.append(f"f {o} {n}")
            model.release(o, n)
            expect.append("freed")
        else:
            n = int(g.integers(1, 2500))
            o = model.alloc(n)
            ops.append(f"a {n}")
            if o is None:
                expect.append("full")
            else:
                live.append((o, n))
                expect.append(f"ok {o}")
        ops.append("s")
        expect.append(f"free {sum(s for _, s in model.free)}")
    got = run(driver, total, ops)
    assert got[: len(expect)] == expect
    # live ranges never overlap
    spans = sorted(live)
    for (a, n), (b, _) in zip(spans, spans[1:]):
        assert a + n <= b


def test_arena_coalesces_back_to_one_block(driver):
    ops = ["a 100", "a 200", "a 300", "f 100 200", "f 0 100", "f 300 300", "a 1000", "s"]
    got = run(driver, 1000, ops)
    assert got[:8] == ["ok 0", "ok 100", "ok 300", "freed", "freed", "freed", "ok 0", "free 0"]


def test_scheduler_under_thread_sanitizer(tmp_path):
    """The quote scheduler's host core (admission by slot and memory, the
    circular scan packing every active quote's blocks into one launch, items
    of one block dealt to one XCD, completion, cancellation, stop) driven by
    a stand-in executor whose "device" thread computes each item with the
    oracle: results alone == in the mix == the oracle over the whole range,
    bit for bit; quotes that a launch finishes reach the executor in one
    batch, each with every block launched; built with -fsanitize=thread, which fails the run on any
    data race between the scheduler, submitting and device threads."""
    csrc = os.path.join(ROOT, "paper_1308_2572_amd", "csrc")
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "sched_driver")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=thread", "-ffp-contract=off", "-c",
                           os.path.join(ROOT, "oracle", "ara_oracle.c"), "-o", obj])
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=thread", "-pthread",
                           "-I", os.path.join(ROOT, "include"), "-I", csrc,
                           os.path.join(ROOT, "tests", "sched_driver.cpp"), os.path.join(csrc, "quote_sched.cpp"),
                           obj, "-o", exe, "-lm"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all scheduler checks passed" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
