"""The serving session's admission policy, on the host: the arena allocator and
the queue that admits requests as slots and memory free up (the scheduler
header compiled alone with g++, driven through a small command interpreter)."""

import os
import random
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2504_01358_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = tmp_path_factory.mktemp("sched") / "sched_driver"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "sched_driver.cpp"), "-o", str(exe)], check=True)

    def run(cmds):
        out = subprocess.run([str(exe)], input="\n".join(cmds) + "\n", capture_output=True,
                             text=True, check=True).stdout
        return [line.split() for line in out.splitlines()]
    return run


def test_arena_first_fit_and_coalescing(driver):
    out = driver(["arena 4096 1 0", "alloc 1000", "alloc 1000", "alloc 1000", "alloc 2000",
                  "release 1024", "release 0", "release 2048", "alloc 4096"])
    assert out[:4] == [["alloc", "0"], ["alloc", "1024"], ["alloc", "2048"], ["alloc", "-1"]]
    # a hole in the middle, then merged with its left neighbour, then everything
    assert out[4] == ["free", "2048", "1024"]
    assert out[5] == ["free", "1024", "2048"]
    assert out[6] == ["free", "0", "4096"]
    assert out[7] == ["alloc", "0"]


def test_budget_binds_and_frees(driver):
    kib = 1024
    out = driver(["arena %d 4 4" % (10 * kib)] + ["push %d %d" % (t, 4 * kib) for t in (1, 2, 3, 4)]
                 + ["admit", "state", "finish 0", "admit", "state", "finish 1", "finish 0", "admit",
                    "state"])
    adm = [o for o in out if o[0] == "admit"]
    assert [a[1] for a in adm[:2]] == ["1", "2"]            # two fit in 10 KiB
    assert out[2] == ["state", "2", "2", str(8 * kib), str(2 * kib)]
    assert adm[2][1] == "3"                                 # admitted once one finished
    assert adm[3][1] == "4"
    assert out[-1][:3] == ["state", "1", "0"]


def test_slots_bound_concurrency(driver):
    out = driver(["arena 1000000 2 4", "push 1 10", "push 2 10", "push 3 10", "admit", "state",
                  "finish 1", "admit"])
    assert [o[1] for o in out if o[0] == "admit"] == ["1", "2", "3"]
    assert out[2] == ["state", "2", "1", "512", str(1000000 - 512)]


def test_bounded_bypass(driver):
    k = 1024
    cmds = ["arena %d 8 2" % (8 * k), "push 1 %d" % (6 * k), "admit",
            "push 2 %d" % (6 * k), "push 3 %d" % k, "push 4 %d" % k, "push 5 %d" % k, "admit",
            "state", "finish 0", "admit", "state"]
    out = driver(cmds)
    adm = [o[1] for o in out if o[0] == "admit"]
    # 3 and 4 overtake the blocked 2 (twice at most); 5 must wait behind it
    assert adm[:3] == ["1", "3", "4"]
    assert out[3] == ["state", "3", "2", str(8 * k), "0"]
    assert adm[3:] == ["2"]


def test_strict_fifo_without_bypass(driver):
    k = 1024
    out = driver(["arena %d 8 0" % (8 * k), "push 1 %d" % (6 * k), "push 2 %d" % (6 * k),
                  "push 3 %d" % k, "admit", "finish 0", "admit"])
    assert [o[1] for o in out if o[0] == "admit"] == ["1", "2", "3"]


def test_random_workload_invariants(driver):
    """Random arrivals and completions: memory and slots are never
    over-committed, every request is admitted exactly once, and everything
    is returned at the end."""
    rng = random.Random(5)
    cap, slots = 64 * 1024, 6
    cmds = ["arena %d %d 3" % (cap, slots)]
    n = 400
    for t in range(1, n + 1):
        cmds.append("push %d %d" % (t, rng.choice([300, 2000, 9000, 30000, 64 * 1024])))
        cmds.append("admit")
        cmds.append("state")
        if rng.random() < 0.7:
            cmds.append("finish %d" % rng.randrange(slots))
            cmds.append("admit")
    for _ in range(4 * n):
        cmds += ["finish %d" % s for s in range(slots)] + ["admit"]
    cmds.append("state")
    out = driver(cmds)
    admitted = [int(o[1]) for o in out if o[0] == "admit"]
    assert sorted(admitted) == list(range(1, n + 1))
    for o in out:
        if o[0] == "state":
            assert int(o[1]) <= slots and int(o[3]) <= cap
    assert out[-1] == ["state", "0", "0", "0", str(cap)]
