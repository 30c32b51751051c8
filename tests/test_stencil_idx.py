"""The trace kernels' node-index arithmetic, compiled for the host.

A micro element of the Freudenthal (Kuhn) refinement of a macro simplex is
given by its base cell k and the rank r_x of each axis in the descending
order of the fractional coordinates (Sec. 2.2, the O(1) micro location).
Its vertex a is V_a = k + e(a) with e(a)_x = [r_x < a]; the P2 node on the
edge (a, b) is the midpoint of V_a and V_b, i.e. the point V_a + V_b of the
lattice of resolution 2n; the P1 nodes are the vertices on the lattice of
resolution n.  Lattice points are numbered I(I+1)(I+2)/6 + J(J+1)/2 + K in
3D and I(I+1)/2 + J in 2D (the block layout of one macro).

The kernel computes these indices without forming the points (sums of
per-axis increments chosen by axis rank).  This test takes the kernel's own
functions (stencil_idx with the lattice helpers it uses) out of the HIP
source, compiles them with the host compiler, and compares them with the
definition above on every base cell and axis order of several levels.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2103_02388_amd", "csrc", "mmoc_trace.hip")


def _function(src, name_regex):
    """The text of the first function whose signature matches name_regex,
    with the template line above it, up to its closing brace."""
    m = re.search(name_regex, src)
    assert m, name_regex
    start = src.rfind("\n", 0, m.start()) + 1
    tmpl = src.rfind("template", 0, start)
    if tmpl >= 0 and src[tmpl:start].count("\n") == 1:
        start = tmpl
    depth, i = 0, src.index("{", m.end() - 1)
    while True:
        if src[i] == "{":
            depth += 1
        elif src[i] == "}":
            depth -= 1
            if depth == 0:
                return src[start:i + 1]
        i += 1


HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#define __device__
#define __forceinline__ inline
%(helpers)s
%(stencil)s

static long lat(int dim, long I, long J, long K)
{
    return dim == 3 ? I * (I + 1) * (I + 2) / 6 + J * (J + 1) / 2 + K : I * (I + 1) / 2 + J;
}

template <int DIM, int ORD>
static long check(int m)
{
    // every axis order: ranks r_x, a permutation of 0..DIM-1
    int perms[6][3], np = 0;
    for (int a = 0; a < DIM; ++a)
        for (int b = 0; b < DIM; ++b)
            for (int c = 0; c < (DIM == 3 ? DIM : 1); ++c) {
                if (a == b || (DIM == 3 && (a == c || b == c))) continue;
                perms[np][0] = a; perms[np][1] = b; perms[np][2] = DIM == 3 ? c : 0; ++np;
            }
    long bad = 0;
    // the base cells of a macro of m cells per edge: k0 < m, k0 >= k1 >= k2
    // (the floors of the cumulative Kuhn coordinates)
    for (int k0 = 0; k0 < m; ++k0)
        for (int k1 = 0; k1 <= k0; ++k1)
            for (int k2 = 0; k2 <= (DIM == 3 ? k1 : 0); ++k2)
                for (int p = 0; p < np; ++p) {
                    int k[3] = {k0, k1, k2};
                    int r[3] = {perms[p][0], perms[p][1], perms[p][2]};
                    constexpr int NN = ORD == 2 ? (DIM + 1) * (DIM + 2) / 2 : DIM + 1;
                    int idx[NN];
                    stencil_idx<DIM, ORD>(k, r, idx);
                    int c = 0;
                    auto node = [&](int a, int b) {
                        long x[3];
                        for (int d = 0; d < 3; ++d) {
                            const int ea = d < DIM && r[d] < a, eb = d < DIM && r[d] < b;
                            x[d] = ORD == 2 ? 2L * k[d] + ea + eb : (long)k[d] + ea;
                        }
                        const long want = DIM == 3 ? lat(3, x[0], x[1], x[2]) : lat(2, x[0], x[1], 0);
                        if (idx[c] != want) {
                            if (bad < 5)
                                printf("DIM %%d ORD %%d m %%d k (%%d %%d %%d) r (%%d %%d %%d) node %%d: %%d != %%ld\n", DIM, ORD,
                                       m, k0, k1, k2, r[0], r[1], r[2], c, idx[c], want);
                            ++bad;
                        }
                        ++c;
                    };
                    if (ORD == 1) {
                        for (int a = 0; a <= DIM; ++a) node(a, a);
                    } else {
                        for (int a = 0; a <= DIM; ++a) node(a, a);
                        for (int a = 0; a <= DIM; ++a)
                            for (int b = a + 1; b <= DIM; ++b) node(a, b);
                    }
                }
    return bad;
}

int main()
{
    long bad = 0, levels = 0;
    for (int m = 1; m <= 128; m *= 2, ++levels) {
        bad += check<3, 2>(m) + check<3, 1>(m) + check<2, 2>(m) + check<2, 1>(m);
    }
    printf("levels %%ld mismatches %%ld\n", levels, bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_stencil_idx_matches_the_lattice_definition(tmp_path):
    src = open(SRC).read()
    tri = re.search(r"__device__ __forceinline__ int tri_n\(int x\) \{[^}]*\}", src).group(0)
    tet = re.search(r"__device__ __forceinline__ int tet_n\(int x\) \{[^}]*\}", src).group(0)
    helpers = tri + "\n" + tet
    stencil = _function(src, r"void stencil_idx\(const int\* k, const int\* r, int\* idx\)")
    assert "template <int DIM, int ORD>" in stencil
    cpp = tmp_path / "stencil_idx.cpp"
    cpp.write_text(HARNESS % {"helpers": helpers, "stencil": stencil})
    exe = tmp_path / "stencil_idx"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(cpp)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "mismatches 0" in r.stdout
