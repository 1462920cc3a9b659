"""CPU tests of the render server's host-side admission pieces (the
first-fit byte arena and the FIFO-with-bounded-bypass rule), compiled from
the same header the server uses, against plain Python models."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2408_07967_amd", "csrc")
ALIGN = 256


@pytest.fixture(scope="module")
def driver():
    td = tempfile.mkdtemp(prefix="fgs_arena_")
    exe = os.path.join(td, "arena_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", HDR,
                    os.path.join(ROOT, "tests", "host", "arena_driver.cpp"), "-o", exe], check=True)
    return exe


def run(exe, lines):
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    return r.stdout.strip().splitlines()


class ArenaModel:
    """First fit over free ranges sorted by offset, coalesced on release."""

    def __init__(self, size):
        self.size = size // ALIGN * ALIGN
        self.free = [(0, self.size)] if self.size else []
        self.used = 0

    @staticmethod
    def rnd(n):
        n = (n + ALIGN - 1) // ALIGN * ALIGN
        return n if n else ALIGN

    def alloc(self, n):
        n = self.rnd(n)
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                self.free[i:i + 1] = [(o + n, s - n)] if s > n else []
                self.used += n
                return o
        return None

    def release(self, o, n):
        n = self.rnd(n)
        self.used -= n
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for o2, s2 in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o2:
                merged[-1] = (merged[-1][0], merged[-1][1] + s2)
            else:
                merged.append((o2, s2))
        self.free = merged


def test_arena_matches_first_fit_model(driver):
    rng = np.random.default_rng(1)
    size = 1 << 22
    lines, expect = ["init %d" % size], ["init %d" % size]
    model = ArenaModel(size)
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            i = int(rng.choice(list(live)))
            o, n = live.pop(i)
            model.release(o, n)
            lines.append(f"free {i}")
            expect.append(f"freed {model.used}")
        else:
            n = int(rng.integers(0, 300_000))
            o = model.alloc(n)
            lines.append(f"alloc {step} {n}")
            if o is None:
                expect.append(f"fail {model.used}")
            else:
                live[step] = (o, n)
                expect.append(f"ok {o} {model.used}")
    got = run(driver, lines)
    assert got == expect
    # no two live regions overlap and all lie inside the arena
    spans = sorted((o, o + ArenaModel.rnd(n)) for o, n in live.values())
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 <= b0
    assert not spans or spans[-1][1] <= size


def test_arena_coalesces_back_to_one_range(driver):
    lines = ["init 10000"] + [f"alloc {i} 100" for i in range(39)] + [f"free {i}" for i in (5, 3, 4, 0, 38)]
    lines += [f"free {i}" for i in range(1, 38) if i not in (3, 4, 5)] + ["alloc 99 9984"]
    got = run(driver, lines)
    assert got[0] == "init 9984"
    assert got[-1] == "ok 0 9984"  # every release merged: the whole arena is one range again


def admit_model(max_bypass, free, need, counters):
    admitted, byp, blocked = [], 0, None
    for i, n in enumerate(need):
        if blocked is not None and counters[blocked] >= max_bypass:
            break
        if n > free:
            if blocked is None:
                blocked = i
            continue
        free -= n
        admitted.append(i)
        if blocked is not None:
            counters[blocked] += 1
            byp += 1
    return admitted, byp, counters


def test_bounded_bypass_matches_model(driver):
    rng = np.random.default_rng(2)
    lines, expect = [], []
    for _ in range(400):
        n = int(rng.integers(1, 9))
        need = [int(x) for x in rng.integers(1, 100, n)]
        counters = [int(x) for x in rng.integers(0, 3, n)]
        mb, free = int(rng.integers(0, 4)), int(rng.integers(0, 300))
        lines.append(f"admit {mb} {free} {n} " + " ".join(map(str, need + counters)))
        a, b, c = admit_model(mb, free, need, list(counters))
        expect.append("admitted" + "".join(f" {i}" for i in a) + f" | bypasses {b} | counters" +
                      "".join(f" {x}" for x in c))
    assert run(driver, lines) == expect


def test_fifo_when_bypass_is_zero(driver):
    # head does not fit: nothing behind it may go ahead
    got = run(driver, ["admit 0 50 3 80 10 10 0 0 0"])
    assert got == ["admitted | bypasses 0 | counters 0 0 0"]
    # head fits: strict arrival order
    got = run(driver, ["admit 0 100 3 30 30 30 0 0 0"])
    assert got == ["admitted 0 1 2 | bypasses 0 | counters 0 0 0"]
    # bounded: two later requests overtake the head, the third waits
    got = run(driver, ["admit 2 50 5 80 10 10 10 10 0 0 0 0 0"])
    assert got == ["admitted 1 2 | bypasses 2 | counters 2 0 0 0 0"]
