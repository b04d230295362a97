"""The device index functions of the library (paper_1010_5433_amd/csrc/geom.h:
even/odd site decoding, neighbour indices, staggered phases with the
antiperiodic time boundary, and the XCD-aware workgroup order) compiled for
the host with AddressSanitizer and UndefinedBehaviorSanitizer and with
bounds asserts around every call, then run

  * exhaustively on every lattice with L_mu in {2, 4, 6} and on a few longer
    ones: every site of both parities and every hop stays in [0, V/2),
    lands on the other parity, and equals the eo index computed from the
    shifted coordinates; every sign is the staggered phase times the
    boundary sign computed from the coordinates;
  * on boundary and random sites of lattices up to the largest the library
    accepts (V/2 < 2^30), where an int overflow would show;
  * and xcd_tile is checked to be a bijection of [0, n) for every n up to
    5000 and a few large n, so that every workgroup's tile is covered once.

A CPU build of the kernels' own index code, not a re-implementation: the
source file is included as it is, with the device qualifiers defined away.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1010_5433_amd", "csrc")

PROGRAM = r'''
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <vector>
#define __device__
#define __forceinline__ inline
#include "geom.h"
using namespace stag;

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails++ < 20) { std::fprintf(stderr, __VA_ARGS__); std::fprintf(stderr, "\n"); } } } while (0)

static int64_t eo_of(const int L[4], const int y[4]) {
    const int64_t lex = y[0] + (int64_t)L[0] * (y[1] + (int64_t)L[1] * (y[2] + (int64_t)L[2] * y[3]));
    return lex >> 1;
}

static void check_site(const Geom &g, int p, int i) {
    int x[4];
    site_coords(g, p, i, x);
    for (int mu = 0; mu < 4; ++mu) CHECK(x[mu] >= 0 && x[mu] < g.L[mu], "coord %d out of range at i=%d", mu, i);
    CHECK(((x[0] + x[1] + x[2] + x[3]) & 1) == p, "parity of i=%d", i);
    CHECK(eo_of(g.L, x) == i, "eo index of the coordinates of i=%d", i);
    for (int mu = 0; mu < 4; ++mu) {
        for (int dir = -1; dir <= 1; dir += 2) {
            const int j = site_nbr(g, i, x, mu, dir);
            CHECK(j >= 0 && j < g.Vh, "neighbour out of range: i=%d mu=%d dir=%d j=%d Vh=%d", i, mu, dir, j, g.Vh);
            int y[4] = {x[0], x[1], x[2], x[3]};
            y[mu] = (x[mu] + dir + g.L[mu]) % g.L[mu];
            CHECK(eo_of(g.L, y) == j, "neighbour index: i=%d mu=%d dir=%d", i, mu, dir);
            CHECK(((y[0] + y[1] + y[2] + y[3]) & 1) == 1 - p, "neighbour parity: i=%d mu=%d", i, mu);
        }
        int eta = 1;
        for (int nu = 0; nu < mu; ++nu) eta = (x[nu] & 1) ? -eta : eta;
        const int bf = (g.antiperiodic && mu == 3 && x[3] == g.L[3] - 1) ? -1 : 1;
        const int bb = (g.antiperiodic && mu == 3 && x[3] == 0) ? -1 : 1;
        CHECK(fwd_sign(g, x, mu) == eta * bf, "forward sign i=%d mu=%d", i, mu);
        CHECK(bwd_sign(g, x, mu) == eta * bb, "backward sign i=%d mu=%d", i, mu);
    }
}

int main() {
    long sites = 0;
    std::vector<std::vector<int>> dims;
    const int small[3] = {2, 4, 6};
    for (int a : small) for (int b : small) for (int c : small) for (int d : small) dims.push_back({a, b, c, d});
    dims.push_back({8, 8, 8, 8});
    dims.push_back({32, 4, 2, 2});
    dims.push_back({2, 2, 2, 32});
    dims.push_back({16, 6, 10, 4});
    for (auto &D : dims) {
        for (int ap = 0; ap < 2; ++ap) {
            const Geom g = make_geom(D.data(), ap);
            for (int p = 0; p < 2; ++p)
                for (int i = 0; i < g.Vh; ++i, ++sites) check_site(g, p, i);
        }
    }
    // large lattices: boundary and pseudo-random sites
    const int big[4][4] = {{256, 256, 256, 64}, {64, 64, 64, 1024}, {1024, 512, 32, 64}, {48, 48, 48, 96}};
    uint64_t s = 12345;
    for (auto &B : big) {
        const Geom g = make_geom(B, 1);
        CHECK((int64_t)B[0] * B[1] * B[2] * B[3] / 2 == g.Vh, "Vh of a large lattice");
        for (int p = 0; p < 2; ++p) {
            const int edge[6] = {0, 1, g.Lh0 - 1, g.Lh0, g.Vh - g.Lh0, g.Vh - 1};
            for (int i : edge) { check_site(g, p, i); ++sites; }
            for (int k = 0; k < 20000; ++k) {
                s = s * 6364136223846793005ull + 1442695040888963407ull;
                check_site(g, p, (int)((s >> 33) % (uint64_t)g.Vh));
                ++sites;
            }
        }
    }
    // xcd_tile: a bijection of [0, n)
    std::vector<int> seen;
    std::vector<int> ns;
    for (int n = 1; n <= 5000; ++n) ns.push_back(n);
    ns.push_back(65536); ns.push_back(2048 * 1024 + 7);
    for (int n : ns) {
        seen.assign(n, 0);
        for (int k = 0; k < n; ++k) {
            const int t = xcd_tile(k, n);
            CHECK(t >= 0 && t < n, "xcd_tile(%d, %d) = %d out of range", k, n, t);
            if (t >= 0 && t < n) seen[t]++;
        }
        for (int t = 0; t < n; ++t) CHECK(seen[t] == 1, "xcd_tile: tile %d of %d covered %d times", t, n, seen[t]);
    }
    std::printf("sites %ld fails %d\n", sites, fails);
    return fails ? 1 : 0;
}
'''


def test_device_index_functions_on_the_host(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    src = tmp_path / "geom_check.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "geom_check"
    r = subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        f"-I{CSRC}", str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "fails 0" in r.stdout
    assert "runtime error" not in r.stderr
