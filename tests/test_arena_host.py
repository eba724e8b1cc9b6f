"""Host-only checks of the serving runtime's device-arena sub-allocator and
admission rule (csrc/arena.h, compiled with g++): first fit, 256-byte
granularity, coalescing, exhaustion, and admission by slots and budget."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r'''
#include <cassert>
#include <cstdio>
#include <random>
#include <vector>
#include "arena.h"
using pcg::Arena;
int main() {
    Arena a(4096);
    size_t o1, o2, o3, o4;
    assert(a.size() == 4096);
    assert(a.alloc(100, &o1) && o1 == 0);          // rounded to 256
    assert(a.alloc(256, &o2) && o2 == 256);
    assert(a.alloc(1000, &o3) && o3 == 512);       // 1024 bytes
    assert(a.in_use() == 256 + 256 + 1024);
    assert(!a.alloc(4096, &o4));                  // does not fit
    assert(a.release(o2) && !a.release(o2));      // double release rejected
    assert(a.alloc(200, &o4) && o4 == 256);       // first fit reuses the hole
    assert(a.release(o1) && a.release(o4) && a.release(o3));
    assert(a.in_use() == 0 && a.free_blocks() == 1 && a.largest_free() == 4096);  // coalesced
    // random alloc/free never overlaps and always coalesces back
    std::mt19937 rng(7);
    Arena b(1 << 20);
    std::vector<std::pair<size_t, size_t>> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || (rng() % 3 != 0)) {
            size_t len = 1 + rng() % 20000, off;
            if (b.alloc(len, &off)) {
                size_t r = Arena::round(len);
                for (auto& l : live) assert(off + r <= l.first || l.first + l.second <= off);
                assert(off + r <= b.size());
                live.push_back({off, r});
            }
        } else {
            size_t k = rng() % live.size();
            assert(b.release(live[k].first));
            live.erase(live.begin() + k);
        }
    }
    for (auto& l : live) assert(b.release(l.first));
    assert(b.in_use() == 0 && b.free_blocks() == 1);
    // admission: slots and budget
    assert(pcg::admissible(100, 0, 60, 0, 2));
    assert(!pcg::admissible(100, 60, 60, 1, 2));     // over budget
    assert(pcg::admissible(100, 40, 60, 1, 2));
    assert(!pcg::admissible(100, 0, 60, 2, 2));      // no free slot
    assert(!pcg::admissible(100, 0, 101, 0, 2));     // larger than the budget
    printf("ok\n");
    return 0;
}
'''


def test_arena_allocator_and_admission(tmp_path):
    src = tmp_path / "arena_test.cpp"
    src.write_text(PROG)
    exe = tmp_path / "arena_test"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-UNDEBUG",
                           "-I" + os.path.join(ROOT, "paper_1302_7193_amd", "csrc"),
                           str(src), "-o", str(exe)])
    assert subprocess.check_output([str(exe)]).strip() == b"ok"
