"""CPU tests of the library's arena allocator (the device-memory bookkeeping
behind admission in batch and serving), built from its own header with the
host compiler and compared with a brute-force first-fit model."""
import os
import random
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ALIGN = 256


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = tmp_path_factory.mktemp("arena") / "arena"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I",
                    os.path.join(ROOT, "paper_1803_03797_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "arena_harness.cpp"), "-o", str(exe)],
                   check=True)
    return str(exe)


def run(exe, script):
    out = subprocess.run([exe], input=script, capture_output=True, text=True, check=True)
    return out.stdout.split("\n")


class Model:
    """Brute force: a byte map of the region, first fit by address scan."""

    def __init__(self, size):
        self.blocks = size // ALIGN
        self.used = [False] * self.blocks
        self.live = {}

    def alloc(self, n):
        k = max(1, -(-max(n, 1) // ALIGN))
        run_start, run_len = 0, 0
        for i in range(self.blocks):
            if self.used[i]:
                run_start, run_len = i + 1, 0
                continue
            run_len += 1
            if run_len == k:
                for j in range(run_start, run_start + k):
                    self.used[j] = True
                return run_start * ALIGN, k
        return -1, 0

    def state(self):
        in_use = sum(self.used) * ALIGN
        runs, cur = [], 0
        for u in self.used + [True]:
            if u:
                if cur:
                    runs.append(cur)
                cur = 0
            else:
                cur += 1
        return in_use, max(runs, default=0) * ALIGN, len(runs)


@pytest.mark.parametrize("seed", range(6))
def test_matches_first_fit_model(harness, seed):
    rng = random.Random(seed)
    size = rng.choice([64 * ALIGN, 1000 * ALIGN + 17, 333 * ALIGN])
    m = Model(size)
    lines, expect, live = ["init %d" % size], [], {}
    for op in range(400):
        if live and rng.random() < 0.45:
            i = rng.choice(sorted(live))
            off, k = live.pop(i)
            for j in range(off // ALIGN, off // ALIGN + k):
                m.used[j] = False
            lines.append("r %d" % i)
        else:
            n = rng.choice([1, 255, 256, 257, 3 * ALIGN, rng.randint(1, 40 * ALIGN)])
            off, k = m.alloc(n)
            if off >= 0:
                live[op] = (off, k)
            lines.append("a %d %d" % (op, n))
            expect.append(str(off))
        if op % 37 == 0:
            lines.append("q")
            expect.append("%d %d %d" % m.state())
    lines.append("q")
    expect.append("%d %d %d" % m.state())
    got = run(harness, "\n".join(lines) + "\n")
    assert got[:len(expect)] == expect


def test_full_release_coalesces_and_refusal(harness):
    size = 10 * ALIGN
    script = ["init %d" % size] + ["a %d %d" % (i, ALIGN) for i in range(10)] + ["a 99 1", "q"]
    script += ["r %d" % i for i in (1, 3, 5, 7, 9, 0, 2, 4, 6, 8)] + ["q", "a 100 %d" % size, "q"]
    got = run(harness, "\n".join(script) + "\n")
    assert got[:10] == [str(i * ALIGN) for i in range(10)]
    assert got[10] == "-1"                       # full: refused
    assert got[11] == "%d 0 0" % size            # all in use, no free block
    assert got[12] == "0 %d 1" % size            # every release coalesced into one block
    assert got[13] == "0"                        # the whole region in one allocation
    assert got[14] == "%d 0 0" % size


def test_release_of_unknown_pointer_is_ignored(harness):
    got = run(harness, "init 4096\na 1 100\nr 7\nr 1\nr 1\nq\n")
    assert got[0] == "0" and got[1] == "0 4096 1"
