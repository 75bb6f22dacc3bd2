"""Host-only test of the server's first-fit arena allocator (au_arena.h),
built with g++ (no HIP) and compared with a simple reference model: first
fit in address order over 256-byte granules, merging freed neighbours."""
import os
import random
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1507_07733_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host", "arena_driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("arena") / "arena_driver")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-I" + CSRC,
                           DRIVER, "-o", exe])
    return exe


class Model:
    def __init__(self, size):
        self.size = size & ~255
        self.used = {}          # offset -> bytes

    def alloc(self, n):
        n = max(1, n)
        n = (n + 255) & ~255
        pos = 0
        for o in sorted(self.used):
            if o - pos >= n:
                break
            pos = o + self.used[o]
        if pos + n > self.size:
            return None
        self.used[pos] = n
        return pos

    def free(self, o):
        del self.used[o]

    def in_use(self):
        return sum(self.used.values())


def run(driver, lines):
    out = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    return out.stdout.split("\n")


def test_first_fit_merge_and_accounting(driver):
    rng = random.Random(5)
    size = 1 << 20
    model = Model(size)
    cmds = ["init %d" % size]
    expect = ["ok"]
    live = []
    peak = 0
    for step in range(3000):
        if live and rng.random() < 0.45:
            o, n = live.pop(rng.randrange(len(live)))
            model.free(o)
            cmds.append("free %d %d" % (o, n))
            expect.append("ok")
        else:
            n = rng.choice([1, 100, 256, 257, 4000, 30000, 100000])
            o = model.alloc(n)
            cmds.append("alloc %d" % n)
            if o is None:
                expect.append("full")
            else:
                expect.append("ok %d" % o)
                live.append((o, n))
        peak = max(peak, model.in_use())
        if step % 97 == 0:
            cmds.append("stat")
            expect.append("%d %d %d" % (model.in_use(), peak, size))
    got = run(driver, cmds)
    assert got[:len(expect)] == expect


def test_exhaustion_and_full_release(driver):
    size = 64 * 256
    cmds = ["init %d" % size] + ["alloc 256"] * 65 + ["stat"]
    for i in range(64):
        cmds.append("free %d 256" % (i * 256))
    cmds += ["stat", "alloc %d" % size, "stat"]
    got = run(driver, cmds)
    assert got[1:65] == ["ok %d" % (i * 256) for i in range(64)]
    assert got[65] == "full"
    assert got[66] == "%d %d %d" % (size, size, size)
    assert got[131] == "0 %d %d" % (size, size)
    assert got[132] == "ok 0"
