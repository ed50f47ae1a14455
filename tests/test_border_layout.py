"""Host-side check of the cross-tile inbox layout (`pmf_border.h`): for every
tile shape and connectivity the library uses, each (border pixel, arc leaving
the tile) pair has its own word, the inverse map returns the pair, and the
only words no pair uses are the column words of the corner diagonals (stored
in the rows).  The header is compiled with the host compiler."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1509_06004_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <set>
#include "pmf_border.h"
using namespace pmf;
template <int K, int TW, int TH> int check() {
    using B = Border<K, TW, TH>;
    std::set<int> used;
    int pairs = 0;
    for (int by = 0; by < TH; ++by)
        for (int bx = 0; bx < TW; ++bx)
            for (int k = 0; k < K; ++k) {
                const int nx = bx + DXk(k), ny = by + DYk(k);
                if (nx >= 0 && nx < TW && ny >= 0 && ny < TH) continue;
                ++pairs;
                const int i = B::index(bx, by, k);
                if (i < 0 || i >= B::E || !used.insert(i).second) return 1;
                int x, y, kk;
                B::pair(i, x, y, kk);
                if (x != bx || y != by || kk != k) return 2;
            }
    int unused = 0;
    for (int i = 0; i < B::E; ++i) {
        if (used.count(i)) continue;
        ++unused;
        int x, y, kk;
        B::pair(i, x, y, kk);
        const bool corner = (x == 0 || x == TW - 1) && (y == 0 || y == TH - 1);
        if (!corner || DXk(kk) == 0 || DYk(kk) == 0) return 3;  // only corner diagonals
    }
    if (unused != (K == 4 ? 0 : 4)) return 4;
    if (B::E != border_words(K, TW, TH)) return 5;
    printf("K%d %dx%d E=%d pairs=%d unused=%d\n", K, TW, TH, B::E, pairs, unused);
    return 0;
}
int main() {
    int rc = check<4, 32, 32>();
    if (!rc) rc = check<8, 32, 32>();
    if (!rc) rc = check<4, 64, 16>();
    if (!rc) rc = check<8, 64, 16>();
    return rc;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_border_words_are_a_bijection(tmp_path):
    src = tmp_path / "border_check.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "border_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 4
    assert "K4 32x32 E=128 pairs=128 unused=0" in lines
    assert "K8 32x32 E=384 pairs=380 unused=4" in lines
