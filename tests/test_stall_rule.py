"""The CG driver's stagnation rule and precision ladder (host code, no GPU).

csrc/stall.hpp is plain C++: it is compiled here with g++ into a small
driver that feeds residual histories through the rule and prints what it
decides, so the rule is checked without a GPU.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_17898_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include "stall.hpp"
using namespace mfgp;

// First iteration (checked every `every`) at which the rule ends the cycle
// for the history rr(it), or -1 within `len` iterations.
template <class F> int first_stall(F rr, int len, int every) {
    StallTracker s;
    s.begin(0, rr(0));
    for (int it = every; it <= len; it += every)
        if (s.update(it, rr(it))) return it;
    return -1;
}

int main() {
    // steady geometric convergence: never stalls
    std::printf("%d\n", first_stall([](int it) { return std::pow(0.97, it); }, 20000, 1));
    // convergence, then a flat floor from iteration 300: stalls 100 iterations
    // after the last new minimum
    std::printf("%d\n", first_stall([](int it) { return std::pow(0.8, std::min(it, 300)); }, 20000, 1));
    // the same floor reached at iteration 2000: the window is a quarter of the cycle
    std::printf("%d\n", first_stall([](int it) { return std::pow(0.995, std::min(it, 2000)); }, 20000, 1));
    // oscillating but decreasing by 2x every 150 iterations: never stalls
    std::printf("%d\n", first_stall([](int it) {
        return std::pow(0.5, it / 150.0) * (1.0 + 0.8 * std::sin(0.37 * it)); }, 20000, 1));
    // checks every 8 iterations: the stall is seen at the first check past the window
    std::printf("%d\n", first_stall([](int it) { return std::pow(0.8, std::min(it, 300)); }, 20000, 8));
    // the residual first rises 12.7x and stays there for 1000 iterations,
    // then converges: never ends the cycle while above its start
    std::printf("%d\n", first_stall([](int it) {
        return it < 1000 ? 161.0 : 161.0 * std::pow(0.97, it - 1000); }, 20000, 1));
    // falls twofold and stays flat: not armed (no tenfold fall), never stalls
    std::printf("%d\n", first_stall([](int it) { return it < 10 ? 1.0 : 0.25; }, 20000, 1));
    // falls to 1e-6 by iteration 200, then jumps above its start and stays:
    // no stall while above the start
    std::printf("%d\n", first_stall([](int it) { return it < 200 ? std::pow(0.933, it) : 2.0; }, 20000, 1));
    // the ladder
    std::printf("%d %d %d %d %d %d %d\n", more_accurate_precision(MFGP_BF16X1),
                more_accurate_precision(MFGP_BF16X2), more_accurate_precision(MFGP_BF16X3),
                more_accurate_precision(MFGP_FP32), more_accurate_precision(MFGP_FP32_GRAM),
                more_accurate_precision(MFGP_FP32_DIRECT), more_accurate_precision(MFGP_FP32_VALU));
    // cycle judgements
    std::printf("%d %d %d %d %d %d\n", cycle_wants_fallback(false, 1.0, 1e-5, 1e-6),
                cycle_wants_fallback(false, 3e-6, 2.5e-6, 1e-6), cycle_wants_fallback(false, 2e-6, 1.3e-6, 1e-6),
                cycle_wants_fallback(true, 1.0, 1e-5, 1e-6), cycle_gave_nothing(2e-6, 2e-6),
                cycle_gave_nothing(2e-6, 1.9e-6));
    std::printf("%d\n", cycle_wants_fallback(false, 1.0, NAN, 1e-6));
    // a floor far above tol: two more cycles of the same reduction would not reach it
    std::printf("%d %d %d %d %d\n", cycle_wants_fallback(false, 1.0, 1.5e-2, 1e-6),
                cycle_wants_fallback(false, 1.0, 8e-3, 1e-6), cycle_wants_fallback(false, 1e-2, 1.5e-3, 1e-6),
                cycle_wants_fallback(false, 1.0, 0.05, 1e-6), cycle_wants_fallback(false, 1.0, 1.5e-3, 1e-6));
    // progress reports: the worst recurrence over the columns still iterating
    std::printf("%.3f %.3f\n", worst_recurrence({0, 1, 0}, {4.0, 1.0, 9.0}, {1.0, 1.0, 1.0}),
                worst_recurrence({0, 0, 0}, {4.0, 1.0, 9.0}, {1.0, 1.0, 1.0}));
    return 0;
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("stall")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")


def test_steady_convergence_never_stalls(results):
    assert results[0] == "-1"
    assert results[3] == "-1"


def test_floor_ends_the_cycle_after_the_window(results):
    # a new minimum every iteration up to 300 (0.8 < 0.9), then flat: the
    # window of 100 ends the cycle at 400
    assert results[1] == "400"
    # 0.995^k makes a new minimum (below 0.9 of the best) every 22 iterations
    # up to 2000; the last is 1980, and the window is then max(100, floor(it / 4)):
    # first met where it - 1980 >= floor(it / 4), i.e. it = 2639
    assert 0.995 ** 21 > 0.9 > 0.995 ** 22
    assert results[2] == "2639"
    # checked every 8 iterations: last minimum seen at 304, stop at the first
    # check at least 100 later
    assert results[4] == "408"


def test_no_stall_in_a_rise_or_without_a_tenfold_fall(results):
    assert results[5] == "-1"
    assert results[6] == "-1"
    assert results[7] == "-1"


def test_precision_ladder(results):
    x1, x2, x3, fp32, gram, direct, valu = (int(v) for v in results[8].split())
    assert (x1, x2, x3, fp32, gram, direct, valu) == (2, 4, 5, 5, 5, -1, -1)


def test_cycle_judgements(results):
    # no fallback after a cycle that cut the true residual >= 1/0.7x; fallback
    # after a stagnated cycle or one that did not; give up only when nothing
    # at all was gained
    assert results[9].split() == ["0", "1", "0", "1", "1", "0"]
    assert results[10] == "1"   # a non-finite residual never counts as progress


def test_cycle_judgement_of_a_high_floor(results):
    # 1 -> 1.5e-2: two repeats would end at 3.4e-6 > 1e-6, take the next form;
    # 1 -> 8e-3: two repeats reach 5.1e-7, refine on the same form;
    # 1e-2 -> 1.5e-3: two repeats reach 3.4e-5, take the next form;
    # 1 -> 0.05 (an inexact form's floor): take the next form;
    # 1 -> 1.5e-3: refine on the same form
    assert results[11].split() == ["1", "0", "1", "1", "0"]


def test_progress_reports_the_live_columns(results):
    # a stopped column keeps its last norm (3.0 here); the report shows the
    # columns still iterating (1.0), or every column when none is
    assert results[12].split() == ["1.000", "3.000"]
