"""The worklist and termination protocol (paper §IV-A, §IV-C) as a CPU model under
ThreadSanitizer: threads play workgroups, with the device's ring of lap tickets, reservation
count, oldest-entry donation and outstanding-work counter, over seeded imbalanced trees, with
random pauses between protocol steps. Invariants checked by the model: no node lost, none taken
twice, no data race on the node words (ThreadSanitizer), counters back at zero and every ring
slot free for its next lap at the end. Two planted protocol mistakes show the checks bite."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "worklist_model", "worklist_model.cpp")
ENV = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66")


def build(tmp, mutation=0):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not installed")
    out = os.path.join(tmp, f"worklist_model_{mutation}")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=thread",
           f"-DVC_MODEL_MUTATION={mutation}", SRC, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return out


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    return build(str(tmp_path_factory.mktemp("wm")))


def run(binary, *args):
    return subprocess.run([binary, *map(str, args)], capture_output=True, text=True,
                          timeout=300, env=ENV)


# threads, ring capacity, donation threshold, instances, tree depth, seed
CASES = [
    (2, 8, 2, 1, 16, 1),      # tiny ring: many laps per slot
    (4, 16, 4, 2, 18, 2),
    (8, 32, 8, 3, 18, 3),
    (8, 64, 48, 4, 17, 4),    # high threshold: most branchings donate
    (16, 64, 16, 6, 17, 5),
    (16, 32, 0, 5, 16, 6),    # threshold 0: no donation, roots only
    (12, 128, 96, 2, 19, 7),
    (3, 8, 1, 8, 15, 8),
]


@pytest.mark.parametrize("case", CASES, ids=[f"t{c[0]}_cap{c[1]}_thr{c[2]}" for c in CASES])
def test_protocol_loses_nothing_and_has_no_data_race(model, case):
    r = run(model, *case)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-2000:]
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok ")


def test_missing_work_count_is_caught(tmp_path):
    """A producer that does not count the node it donates as outstanding work: the counter
    goes below zero when the sub-tree is released."""
    r = run(build(str(tmp_path), 1), 8, 64, 8, 3, 16, 1)
    assert r.returncode == 1 and "below zero" in r.stderr


def test_relaxed_publish_is_a_data_race(tmp_path):
    """A slot published with a relaxed store: ThreadSanitizer reports the race on the node
    words."""
    r = run(build(str(tmp_path), 2), 8, 64, 8, 3, 16, 1)
    assert "ThreadSanitizer: data race" in r.stderr
