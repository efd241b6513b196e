"""Host-only check of the first-phase merge's index arithmetic (Alg. 3, union of the first
trees' leaves): every slot, leaf-start and permutation read the merge kernel makes stays
inside its buffer, for the shapes the GPU tests and the benchmark run.  The replay compiles
the library's own geometry header with g++ (no GPU, no HIP).

The `k_above_leaf` shape (K above the distinct candidates of the first-phase leaves, so the
row threshold is +inf) once read past the row's slots; the replay of the arithmetic before
that fix must fail there, which shows the check can see the fault."""

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "merge_index_replay.cpp")


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("replay") / "merge_index_replay")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-o", exe, SRC])
    return exe


SHAPES = [
    # n, T, n0, K, rows
    (2000, 3, 30, 60, 2000),          # k_above_leaf: tau = +inf on every row
    (40, 2, 4, 3, 40),                # tiny
    (10_000, 4, 50, 10, 10_000),      # 10k x 16 mixture
    (7800, 4, 256, 20, 7800),         # leaves of 243/244 (the 1M-point shape in small)
    (12_000, 12, 200, 100, 12_000),   # K 100
    (8000, 24, 40, 20, 8000),         # many trees
    (1_000_000, 32, 256, 20, 1_000_000),   # 1M x 128, T 32
    (1_000_000, 80, 256, 20, 1_000_000),   # the same forest grown to T 80
    (1_000_000, 48, 512, 10, 1_000_000),   # 1M x 784, n0 512
    (4_000_000, 64, 256, 100, 4096),        # 4M served forest, a batch of queries
    (4_000_000, 64, 256, 1, 1),
    (1_000_000, 80, 256, 20, 1_000_000, "--B", 8),   # bf16 / fp16 over 64+ trees: 8 first trees
    (12_000, 64, 50, 20, 12_000, "--B", 8),
    (100_000, 48, 512, 10, 100_000, "--B", 2),       # the plan tuner's smallest choice
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{s[0]}_T{s[1]}_n0{s[2]}_K{s[3]}" + (f"_B{s[6]}" if len(s) > 5 else "")
                                          for s in SHAPES])
def test_merge_reads_in_range(replay, shape):
    r = subprocess.run([replay, *map(str, shape)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout.splitlines()[-1]


def test_old_arithmetic_is_caught(replay):
    # before the fix every lane read Q slot columns, one past the row's three
    r = subprocess.run([replay, "2000", "3", "30", "60", "2000", "--old"], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 1 and "FAIL" in r.stdout
