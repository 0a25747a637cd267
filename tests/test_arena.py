"""Host-only test of the serving form's arena allocator (rp_arena.h): random
allocate/free sequences never hand out overlapping or out-of-range blocks,
the byte accounting matches, an allocation fails only when no free block is
large enough, and freeing everything coalesces back to one block."""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2103_01216_amd", "csrc")

DRIVER = r'''
#include "rp_arena.h"
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include <algorithm>
struct Blk { uint64_t off, bytes; };
int main(int argc, char **argv) {
    const uint64_t size = strtoull(argv[1], 0, 10);
    const unsigned seed = (unsigned)atoi(argv[2]);
    const int steps = atoi(argv[3]);
    std::mt19937_64 rng(seed);
    rpserve::Arena a;
    a.reset(size);
    std::vector<Blk> live;
    uint64_t used = 0;
    for (int s = 0; s < steps; s++) {
        if (!live.empty() && (rng() % 100) < 45) {
            size_t i = rng() % live.size();
            a.free(live[i].off, live[i].bytes);
            used -= rpserve::Arena::rounded(live[i].bytes);
            live.erase(live.begin() + i);
        } else {
            uint64_t bytes = 1 + rng() % (size / 8);
            if (rng() % 4 == 0) bytes = 1 + rng() % 300;
            uint64_t off;
            const bool ok = a.alloc(bytes, &off);
            if (!ok) {
                if (a.largest_free() >= rpserve::Arena::rounded(bytes)) { puts("FAIL spurious"); return 1; }
                continue;
            }
            if (off % rpserve::ALIGN || off + bytes > size) { puts("FAIL range"); return 1; }
            for (auto &b : live)
                if (off < b.off + b.bytes && b.off < off + bytes) { puts("FAIL overlap"); return 1; }
            live.push_back({off, bytes});
            used += rpserve::Arena::rounded(bytes);
        }
        if (a.in_use() != used) { puts("FAIL accounting"); return 1; }
        if (a.peak() < a.in_use()) { puts("FAIL peak"); return 1; }
    }
    for (auto &b : live) a.free(b.off, b.bytes);
    if (a.in_use() != 0 || a.free_blocks() != 1 || a.largest_free() != size) { puts("FAIL coalesce"); return 1; }
    puts("OK");
    return 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("arena")
    src = d / "arena_driver.cpp"
    src.write_text(DRIVER)
    exe = d / "arena_driver"
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe), str(src)])
    return str(exe)


@pytest.mark.parametrize("size,seed", [(1 << 20, 1), (1 << 20, 2), (64 << 30, 3), (4096, 4),
                                       (1000 * 256, 5)])
def test_random_sequences(driver, size, seed):
    out = subprocess.run([driver, str(size), str(seed), "20000"], capture_output=True,
                         text=True, timeout=120)
    assert out.stdout.strip() == "OK", out.stdout
