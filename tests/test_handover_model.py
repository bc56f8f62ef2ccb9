"""CPU: the search kernel's work hand-over (Sec. V-A), run as a host model.

tests/handover_model.cpp plays each wavefront with a host thread that runs
the kernel's search loop over a synthetic search tree, with the kernel's own
split rules and task record (csrc/handover.h) and its claim / mailbox /
termination protocol on std::atomic.  Checked here:
  * no work lost or duplicated: the matches found (count, sum and xor of
    their ids) equal a sequential traversal of the same tree, under forced
    and probabilistic hand-over, 2 to 64 threads, every kind of split
    (candidate ranges, chunk survivors, core permutations) exercised;
  * every work item ends: the pending count and every seed's open-item
    counter (the per-update completion report) return to 0;
  * no data races (ThreadSanitizer build);
  * progress: a rule that hands on a single core permutation does not
    terminate (a wave that receives one polls before entering it and hands
    it on again), while the kernel's rule, under which the donor keeps at
    least one unit, terminates with few hand-overs."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "handover_model.cpp")


def _build(out_dir, name, extra):
    exe = os.path.join(str(out_dir), name)
    r = subprocess.run(["g++", "-std=c++17", "-pthread", "-Wall", "-o", exe, SRC] + extra,
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-4000:])
    return exe


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    return _build(tmp_path_factory.mktemp("ho"), "model", ["-O2"])


def _run(exe, threads, seeds, forced, perms_rule=0, cap=0, salt=1, scenario=0, timeout=120):
    r = subprocess.run([exe, str(threads), str(seeds), str(int(forced)), str(perms_rule), str(cap), str(salt),
                        str(scenario)], capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, r.stderr[-3000:]
    f = r.stdout.split()
    v = {f[i]: f[i + 1] for i in range(0, len(f) - 1) if not f[i].lstrip("-").isdigit()}
    out = {"matches": int(f[1]), "sum": int(f[3]), "xor": int(f[5]),
           "ho": (int(f[7]), int(f[8]), int(f[9])), "ref": (int(f[11]), int(f[12]), int(f[13])),
           "closed": int(v["closed"]), "pending": int(v["pending"]), "stalled": int(v["stalled"]),
           "stderr": r.stderr}
    return out


def _exact(o):
    assert o["stalled"] == 0
    assert (o["matches"], o["sum"], o["xor"]) == o["ref"]
    assert o["closed"] == 1 and o["pending"] == 0


@pytest.mark.parametrize("threads,seeds,forced,salt", [
    (2, 200, True, 1), (8, 200, True, 2), (16, 300, False, 3), (32, 200, True, 4), (64, 400, True, 5),
    (64, 400, False, 6), (12, 50, True, 7),
])
def test_no_work_lost_or_duplicated(model, threads, seeds, forced, salt):
    o = _run(model, threads, seeds, forced, salt=salt)
    _exact(o)
    assert o["ref"][0] > 0


def test_every_kind_of_split_is_handed_over(model):
    """Which kinds of work a run hands over depends on thread timing; over a
    few forced runs, candidate ranges, chunk survivors and core permutations
    must each have been handed over, every run exact."""
    seen = [0, 0, 0]
    for salt in range(11, 19):
        o = _run(model, 16, 300, True, salt=salt)
        _exact(o)
        seen = [a + b for a, b in zip(seen, o["ho"])]
        if all(h > 0 for h in seen):
            break
    assert all(h > 0 for h in seen), seen


def test_under_thread_sanitizer(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    try:
        exe = _build(tmp_path, "model_tsan", ["-O1", "-g", "-fsanitize=thread"])
    except RuntimeError as e:
        pytest.skip("no ThreadSanitizer runtime: %s" % str(e)[:200])
    for threads, seeds, forced, salt in ((16, 300, True, 7), (32, 300, False, 8)):
        o = _run(exe, threads, seeds, forced, salt=salt, timeout=300)
        assert "ThreadSanitizer" not in o["stderr"], o["stderr"][-3000:]
        _exact(o)


@pytest.mark.parametrize("threads", [8, 32])
def test_handing_on_a_single_permutation_does_not_terminate(model, threads):
    """One seed whose core has three valid permutations: the first split hands
    one of them to an idle wave.  Handing on a single permutation then passes
    it from idle wave to idle wave without end: with one such chain every
    claim finds an idle wave (the previous holder advertises itself again),
    so the search never ends.  (With several chains two holders can race for
    the same idle bits, and a holder that claims none enters the permutation
    itself, so there the pre-fix rule only usually livelocks.)"""
    cap = 20000
    bad = _run(model, threads, 1, True, perms_rule=1, cap=cap, salt=3, scenario=1)
    assert bad["stalled"] == 1 and bad["ho"][2] > cap


@pytest.mark.parametrize("threads,seeds", [(8, 1), (8, 2), (32, 4)])
def test_kernel_rule_enters_a_single_handed_permutation(model, threads, seeds):
    """The same scenario with the kernel's rule: a wave that receives a single
    permutation enters it, so the search ends with the exact result after a
    handful of permutation hand-overs."""
    good = _run(model, threads, seeds, True, perms_rule=0, cap=20000, salt=3, scenario=1)
    _exact(good)
    assert 0 < good["ho"][2] < 100
