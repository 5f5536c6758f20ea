"""CPU test of the solve server's HBM-arena allocator (host-only header, built
with g++): first fit, coalescing, admission of a FIFO request stream within the
budget, and no overlap between live allocations."""
import os
import subprocess

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "mg_arena.h"
int main() {
    mgrt::Arena a;
    a.reset(1000 * 256 + 17);            // rounded down to whole 256-byte units
    if (a.size() != 1000 * 256 || a.free_bytes() != a.size()) return 1;
    size_t o1, o2, o3, o4;
    if (!a.alloc(300 * 256, &o1) || o1 != 0) return 2;
    if (!a.alloc(100 * 256 + 1, &o2) || o2 != 300 * 256) return 3;   // rounded up to 101 units
    if (!a.alloc(500 * 256, &o3) || o3 != 401 * 256) return 4;
    if (a.alloc(100 * 256, &o4)) return 5;                           // only 99 units left
    a.release(o2, 100 * 256 + 1);
    if (!a.alloc(50 * 256, &o4) || o4 != 300 * 256) return 6;        // first fit reuses the hole
    a.release(o1, 300 * 256);
    a.release(o4, 50 * 256);
    a.release(o3, 500 * 256);
    if (a.fragments() != 1 || a.free_bytes() != a.size()) return 7;  // everything coalesced
    // random FIFO admission stream: requests wait until they fit, live ranges never overlap
    std::srand(7);
    std::vector<std::pair<size_t, size_t>> live;
    size_t admitted = 0, peak = 0;
    for (int step = 0; step < 20000; step++) {
        size_t want = (size_t)(1 + std::rand() % 200) * 256;
        size_t off;
        if (a.alloc(want, &off)) {
            for (auto& l : live)
                if (off < l.first + l.second && l.first < off + want) return 8;
            if (off + want > a.size()) return 9;
            live.push_back({off, want});
            admitted++;
        } else if (!live.empty()) {
            size_t k = std::rand() % live.size();
            a.release(live[k].first, live[k].second);
            live.erase(live.begin() + k);
        }
        size_t used = a.size() - a.free_bytes();
        peak = used > peak ? used : peak;
        size_t sum = 0;
        for (auto& l : live) sum += l.second;
        if (sum != used) return 10;
    }
    std::printf("%zu %zu\n", admitted, peak);
    return 0;
}
'''


def test_arena_first_fit_and_budget(tmp_path):
    src = tmp_path / "arena_test.cpp"
    exe = tmp_path / "arena_test"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-I",
                    os.path.join(ROOT, "paper_1410_8568_amd", "csrc"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, f"arena check {out.returncode} failed"
    admitted, peak = map(int, out.stdout.split())
    assert admitted > 1000 and peak <= 1000 * 256
