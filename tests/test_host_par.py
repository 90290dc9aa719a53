"""The host analysis's fork/join helpers (csrc/par.h), compiled with g++ into a
small program: parallel_chunks covers [0, n) once in contiguous ascending
chunks for every size and grain, the chunk indices are distinct and in range,
run_pair runs both tasks, and an exception thrown by a worker (or by the calling
thread) reaches the caller after every worker has joined."""
import os
import shutil
import subprocess
import tempfile

import pytest

from paper_1812_06160_amd import build as B

PROGRAM = r"""
#include "par.h"
#include <atomic>
#include <cstdio>
#include <mutex>
#include <stdexcept>
#include <utility>
#include <vector>
using namespace jv;
static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL %s line %d\n", #c, __LINE__); ++fails; } } while (0)
int main() {
    const int T = host_threads();
    CHECK(T >= 1 && T <= 16);
    for (long long n : {0LL, 1LL, 7LL, 64LL, 1000LL, 16385LL, 1000003LL})
        for (long long grain : {0LL, 1LL, 100LL, 1LL << 14}) {
            std::vector<int> hit((size_t)n, 0);
            std::vector<std::pair<long long, long long>> seen(T, {-1, -1});
            std::mutex m;
            const int nc = parallel_chunks(n, grain, [&](int c, long long lo, long long hi) {
                CHECK(c >= 0 && c < T);
                {
                    std::lock_guard<std::mutex> g(m);
                    CHECK(seen[c].first < 0);
                    seen[c] = {lo, hi};
                }
                for (long long i = lo; i < hi; ++i) hit[(size_t)i]++;
            });
            CHECK(nc >= 1 && nc <= T);
            for (long long i = 0; i < n; ++i) CHECK(hit[(size_t)i] == 1);
            long long at = 0;
            for (int c = 0; c < nc; ++c) {
                CHECK(seen[c].first == at);
                at = seen[c].second;
            }
            CHECK(at == n);
        }
    std::atomic<int> a{0}, b{0};
    run_pair([&] { a = 1; }, [&] { b = 2; });
    CHECK(a == 1 && b == 2);
    int caught = 0;
    try {
        run_pair([] {}, [] { throw std::runtime_error("worker"); });
    } catch (const std::runtime_error &) { caught++; }
    try {
        run_pair([] { throw std::runtime_error("caller"); }, [] {});
    } catch (const std::runtime_error &) { caught++; }
    std::atomic<int> ran{0};
    try {
        parallel_chunks(1000000, 1, [&](int c, long long, long long) {
            ran++;
            if (c == host_threads() - 1) throw std::runtime_error("last chunk");
        });
    } catch (const std::runtime_error &) { caught++; }
    CHECK(caught == 3);
    CHECK(ran == host_threads());
    std::printf(fails ? "FAILED\n" : "OK\n");
    return fails ? 1 : 0;
}
"""


def test_par_helpers():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "par_test.cpp")
        exe = os.path.join(d, "par_test")
        with open(src, "w") as f:
            f.write(PROGRAM)
        r = subprocess.run([gxx, "-O1", "-std=c++17", "-pthread", "-I", B.CSRC, src, "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-2000:]
