"""Host logic of the HBM arena (paper_1407_1785_amd/csrc/arena.h): a
randomised sequence of takes and gives, checked against the invariants of a
first-fit allocator.  Compiled with g++ on the CPU; no device is involved."""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>
#include "arena.h"

int main() {
    tsvd::Arena a;
    const size_t cap = 1 << 24;
    a.reset(reinterpret_cast<char*>(0x100000), cap);
    std::mt19937_64 rng(14071785);
    std::map<size_t, size_t> live;   // offset -> rounded size
    size_t used = 0;
    for (int step = 0; step < 20000; ++step) {
        const bool give = !live.empty() && (rng() % 100) < 45;
        if (give) {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            a.give(it->first, it->second);
            used -= it->second;
            live.erase(it);
        } else {
            const size_t want = 1 + rng() % (cap / 64);
            size_t off = 0;
            const bool ok = a.take(want, &off);
            const size_t r = tsvd::Arena::round(want);
            if (ok) {
                if (off % 256 != 0 || off + r > cap) { std::printf("bad block\n"); return 1; }
                auto nx = live.lower_bound(off);
                if (nx != live.end() && nx->first < off + r) { std::printf("overlap next\n"); return 1; }
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    if (pv->first + pv->second > off) { std::printf("overlap prev\n"); return 1; }
                }
                live[off] = r;
                used += r;
            } else if (used + r <= cap && live.empty()) {
                std::printf("refused on an empty arena\n");
                return 1;
            }
        }
        if (a.used() != used) { std::printf("used mismatch\n"); return 1; }
    }
    for (auto& kv : live) a.give(kv.first, kv.second);
    size_t off = 1;
    if (!a.take(cap, &off) || off != 0 || a.used() != cap) { std::printf("not coalesced\n"); return 1; }
    std::printf("ok\n");
    return 0;
}
"""


def test_arena_first_fit_invariants(tmp_path):
    src = tmp_path / "arena_test.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "arena_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_1407_1785_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
