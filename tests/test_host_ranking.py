"""Host logic: the ranking of the Hankel singular values (csrc/ranking.hpp, shared with the
device SVD kernel) gives a valid permutation for any input, NaN and Inf included, and the
extraction's finiteness test flags them, so a diverged solve ends in CBS_ENONFINITE
instead of a gather through an incomplete permutation.

The header is compiled with g++ under AddressSanitizer and UndefinedBehaviorSanitizer."""
import math
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1709_09347_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host", "ranking_driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("ranking") / "ranking_driver")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=all", "-I", CSRC, DRIVER, "-o", exe], check=True)
    return exe


def _run(exe, vals):
    txt = f"{len(vals)}\n" + " ".join(repr(float(v)) if math.isfinite(v) else
                                      ("nan" if math.isnan(v) else ("inf" if v > 0 else "-inf"))
                                      for v in vals) + "\n"
    r = subprocess.run([exe], input=txt, capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stderr)
    lines = r.stdout.split("\n")
    perm = [int(t) for t in lines[0].split()]
    return perm, lines[1].strip() == "finite 1"


@pytest.mark.parametrize("vals", [
    [3.0, 1.0, 2.0],
    [1.0, 1.0, 1.0, 0.5],                              # ties go by column index
    [2.0, float("nan"), 1.0, float("nan")],            # NaN below every norm
    [float("inf"), 1.0, float("-inf"), 0.0],           # Inf is not finite either
    [float("nan")] * 5,
    [0.0, -0.0, 1e-300, 5e-324],
])
def test_ranking_is_a_permutation(driver, vals):
    perm, finite = _run(driver, vals)
    n = len(vals)
    assert sorted(perm) == list(range(n))
    key = [v if math.isfinite(v) else -1.0 for v in vals]
    ranked = [key[j] for j in perm]
    assert all(ranked[i] >= ranked[i + 1] for i in range(n - 1))
    for i in range(n - 1):   # equal keys keep column order
        if ranked[i] == ranked[i + 1]:
            assert perm[i] < perm[i + 1]
    assert finite == all(math.isfinite(v) for v in vals)


def test_ranking_random_against_numpy(driver):
    rng = np.random.default_rng(5)
    for _ in range(20):
        v = rng.standard_normal(rng.integers(1, 200)) ** 2
        v[rng.random(v.size) < 0.1] = np.nan
        perm, finite = _run(driver, list(v))
        key = np.where(np.isfinite(v), v, -1.0)
        want = sorted(range(v.size), key=lambda j: (-key[j], j))
        assert perm == want
        assert finite == bool(np.all(np.isfinite(v)))
