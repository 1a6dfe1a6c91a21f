"""Host-side check of the step kernels' 32-bit slot offsets (no GPU).

The fast odd, push and adjoint kernels address a population slot as
base + lo[I] + (off + on[I] mod 2^32) (neighbour) or base + lo[I] +
(off + oo[I] mod 2^32) (own slot), with the offsets of lbm_launch.h's tables
for the row's class (free-slip face rows remap the crossing directions) and,
in the in-place array's row-block layout, for the row's place at a block
edge; base includes the row start there (row_start) and off is x times the
element size, while in the canonical arrays of the push and adjoint off is
the cell's byte offset in its slice.  A host program
compiled against the library's own header enumerates, for every row class,
block edge and storage width, on grids from 3x3x3 to ones at the size
limits (canonical slices below 2 GiB, or 512 MiB with free-slip y or z
faces, whose face rows remap directions up to seven slices away; in-place
arrays of tens of GiB), the cells of rows of that class (x-face cells included), and
checks every address the kernels can form against an independent 64-bit
computation of the intended slot: the own slot I of the cell, and slot
opp(I') of the pull source x - c' (c' = c_I with the components mirrored at
the row's free-slip faces zeroed) whenever that source lies in the grid.
Every address must also fall inside the population array.  The adjoint's
and the push's outflow copies (one element further along x) and the push's inflow-cell
store toward x = 1 are covered by the same enumeration, and the choice of
rows per block (row_blocks) is checked against its statement for every ny
up to 5000, and the multiply-high division that splits the step kernels'
wave index against the hardware division.  Also: lbm_create refuses grids
beyond its limit.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_04516_amd", "csrc")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_2607_04516_amd", "liblbm.so")

SRC = r'''
#include "lbm_launch.h"
#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace lbm;

static const int D[19][3] = {{0,0,0},{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1},{1,1,0},{-1,-1,0},
    {1,0,1},{-1,0,-1},{0,1,1},{0,-1,-1},{1,-1,0},{-1,1,0},{1,0,-1},{-1,0,1},{0,1,-1},{0,-1,1}};
static int find(int x, int y, int z) { for (int i = 0; i < 19; i++) if (D[i][0] == x && D[i][1] == y && D[i][2] == z) return i; return -1; }
static int opposite(int i) { return find(-D[i][0], -D[i][1], -D[i][2]); }

static long long errors = 0, checked = 0;
static void fail(const char* what, const Geo& g, int e, int cls, int x, int y, int z, int I, long long got, long long want)
{
    if (errors < 20)
        std::printf("FAIL %s grid %dx%dx%d elem %d class %d cell (%d,%d,%d) dir %d: %lld vs %lld\n", what, g.nx, g.ny,
                    g.nz, e, cls, x, y, z, I, got, want);
    errors++;
}

// Independent element index of (slot s, x, y, z): blocked (R rows per block,
// rows numbered y + nyr z with nyr >= ny a multiple of R) or plain slices (nyr = ny).
struct Layout {
    bool blocked;
    long long S, pitch, nyr, R;
    long long index(int s, int x, int y, int z) const
    {
        const long long row = y + nyr * z;
        if (!blocked) return s * S + row * pitch + x;
        return ((row / R) * 19 + s) * R * pitch + (row % R) * pitch + x;
    }
};

// Every address a kernel forms for the cells of the sampled rows: own slot,
// pull source (with the row's free-slip mirrors), the push's and the
// adjoint's outflow copy one element further along x.
static void check(const Geo& g, const Layout& L, int e, bool adjoint)
{
    const long long total = 19 * L.S * e;
    std::vector<int> xs = {0, 1, 2, 31, 62, 63, 64, 65, g.nx / 2, g.nx - 3, g.nx - 2, g.nx - 1};
    std::vector<int> ys = {0, 1, 2, 7, 8, 15, 16, 31, 32, 33, g.ny / 2, g.ny - 2, g.ny - 1};
    std::vector<int> zs = {0, 1, g.nz / 2, g.nz - 2, g.nz - 1};
    for (int z : zs) for (int y : ys) {
        if (y < 0 || y >= g.ny || z < 0 || z >= g.nz) continue;
        const long long row = y + (long long)g.ny * z;
        const int cls = row_class(g, y, z);
        StepOff O;
        long long rowbase;   // what the kernel adds to the array base before the lane offset
        uint32_t off0;       // lane offset of x = 0
        if (L.blocked) {
            const long long mrow = mem_row(g, y, z);
            if (mrow != y + L.nyr * z) fail("mem_row", g, e, cls, 0, y, z, 0, mrow, y + L.nyr * z);
            O = step_offsets_blocked(g.pitch, g.nyp, g.lrb, e, cls, block_edge(g, mrow));
            rowbase = row_start(g, mrow, e);
            off0 = 0;
        } else {
            O = step_offsets(L.S, L.pitch, g.ny, e, cls);
            rowbase = 0;
            off0 = (uint32_t)(row * L.pitch) * (uint32_t)e;
        }
        const int my = cls / 3, mz = cls % 3;
        for (int x : xs) {
            if (x < 0 || x >= g.nx) continue;
            const uint32_t off = off0 + (uint32_t)x * (uint32_t)e;   // the kernels' 32-bit lane offset
            for (int I = 0; I < 19; I++) {
                checked++;
                const long long own = rowbase + O.lo[I] + (long long)(uint32_t)(off + O.oo[I]);
                const long long own_want = L.index(I, x, y, z) * e;
                if (own != own_want) fail("own", g, e, cls, x, y, z, I, own, own_want);
                if (rowbase + O.even[I] + (long long)off != own_want && L.blocked) fail("own-even", g, e, cls, x, y, z, I, rowbase + O.even[I] + off, own_want);
                if (own < 0 || own + e > total) fail("own-bounds", g, e, cls, x, y, z, I, own, total);
                int cx = D[I][0], cy = D[I][1], cz = D[I][2];
                int jx = cx, jy = cy, jz = cz;
                if ((my == 1 && cy == 1) || (my == 2 && cy == -1)) { jy = -cy; cy = 0; }
                if ((mz == 1 && cz == 1) || (mz == 2 && cz == -1)) { jz = -cz; cz = 0; }
                const int sx = x - cx, sy = y - cy, sz = z - cz;
                if (sx < 0 || sx >= g.nx || sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz) continue;
                const int slot = opposite(find(jx, jy, jz));
                const long long want = L.index(slot, sx, sy, sz) * e;
                const long long nb = rowbase + O.lo[I] + (long long)(uint32_t)(off + O.on[I]);
                if (nb != want) fail("neighbour", g, e, cls, x, y, z, I, nb, want);
                if (rowbase + O.odd[I] + (long long)off != want) fail("fast", g, e, cls, x, y, z, I, rowbase + O.odd[I] + off, want);
                if (nb < 0 || nb + e > total) fail("neighbour-bounds", g, e, cls, x, y, z, I, nb, total);
                if (!L.blocked && D[I][0] == 1 && x == g.nx - 1) {
                    // push and adjoint: the outflow copy of the slot at nx - 2
                    const long long cp = rowbase + O.lo[I] + (long long)(uint32_t)(off + O.on[I] + (uint32_t)e);
                    if (cp != want + e || cp + e > total) fail("outflow-copy", g, e, cls, x, y, z, I, cp, want + e);
                }
            }
        }
    }
}

// row_blocks against its statement for every ny up to 5000: R = 2^k <= 32,
// nyp the next multiple of R, padding at most ny / 16, and no larger R
// that would satisfy the same bound.
static void check_row_blocks()
{
    for (int ny = 1; ny <= 5000; ny++) {
        int lrb = -1, nyp = -1;
        row_blocks(ny, lrb, nyp);
        const long long R = 1ll << lrb;
        bool ok = lrb >= 0 && lrb <= 5 && nyp % R == 0 && nyp >= ny && nyp - ny < R && (nyp - ny) * 16 <= ny;
        if (ok && lrb < 5) {
            const long long R2 = 2 * R, p2 = (ny + R2 - 1) / R2 * R2;
            ok = (p2 - ny) * 16 > ny;
        }
        if (!ok) {
            if (errors < 20) std::printf("FAIL row_blocks ny %d: lrb %d nyp %d\n", ny, lrb, nyp);
            errors++;
        }
        checked++;
    }
}

// The step kernels split their wave index with multiply-high divisions
// (fast_div / fdiv); against the hardware division for every divisor up to
// 5000 and pseudo-random larger ones, at the range edges and at
// pseudo-random dividends over the whole 32-bit range.
static void check_fast_div()
{
    uint64_t s = 0x9e3779b97f4a7c15ull;
    auto next = [&]() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (uint32_t)(s >> 32); };
    std::vector<uint32_t> ds;
    for (uint32_t d = 1; d <= 5000; d++) ds.push_back(d);
    for (int k = 0; k < 2000; k++) {
        const uint32_t d = next() >> (k % 32);
        ds.push_back(d ? d : 1u);
    }
    ds.push_back(0xffffffffu);
    ds.push_back(0x80000000u);
    ds.push_back(0x80000001u);
    for (uint32_t d : ds) {
        const FastDiv f = fast_div(d);
        auto test = [&](uint32_t n) {
            if (fdiv(n, f) != n / d) {
                if (errors < 20) std::printf("FAIL fdiv %u / %u: %u\n", n, d, fdiv(n, f));
                errors++;
            }
            checked++;
        };
        for (uint32_t n : {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu})
            test(n);
        for (int k = 0; k < 100; k++) test(next());
    }
}

int main()
{
    check_row_blocks();
    check_fast_div();
    struct Case { int nx, ny, nz; int face[6]; };
    // face kinds: 0 periodic, 1 inflow, 2 outflow, 3 free-slip, 4 wall
    std::vector<Case> cases = {
        {3, 3, 3, {1, 2, 3, 3, 4, 3}},
        {64, 48, 32, {1, 2, 3, 3, 4, 3}},
        {65, 17, 9, {1, 2, 3, 3, 3, 3}},
        {800, 800, 128, {1, 2, 1, 2, 4, 3}},
        {256, 256, 96, {1, 2, 3, 3, 4, 3}},
        {37, 29, 23, {4, 4, 3, 3, 3, 3}},
        {1024, 1024, 500, {1, 2, 3, 3, 4, 3}},   // free-slip faces: canonical FP32 refused for the push
        {1024, 1024, 127, {1, 2, 3, 3, 4, 3}},   // free-slip faces, canonical FP32 slices just below 512 MiB
        {1024, 1024, 500, {1, 2, 1, 2, 4, 4}},   // no free-slip face: canonical FP32 slices just below 2 GiB
        {4096, 4096, 40, {1, 2, 3, 3, 4, 3}},    // in-place array 48 GiB in FP64
        {805, 897, 160, {1, 2, 1, 2, 4, 3}},     // odd ny: 32-row blocks over 928 padded rows
        {96, 102, 40, {1, 2, 3, 3, 4, 3}},       // a slab with ghost rows: 8-row blocks over 104
    };
    for (const Case& c : cases) {
        for (int e : {8, 4, 2}) {
            Geo g{};
            g.nx = c.nx; g.ny = c.ny; g.nz = c.nz;
            g.ncx = (g.nx + 63) / 64; g.pitch = g.ncx * 64; g.wpr = g.ncx;
            row_blocks(g.ny, g.lrb, g.nyp);
            const long long R = 1ll << g.lrb;
            // padding: whole blocks, at most ny / 16 extra rows, and no smaller
            // padding with a larger block
            if (g.nyp % R != 0 || g.nyp < g.ny || (g.nyp - g.ny) * 16 > g.ny || g.nyp - g.ny >= R) {
                std::printf("FAIL row blocks ny %d: lrb %d nyp %d\n", g.ny, g.lrb, g.nyp);
                errors++;
            }
            for (int k = 0; k < 6; k++) g.face[k] = c.face[k];
            g.S = (long long)g.pitch * g.nyp * g.nz;
            g.N = (long long)g.nx * g.ny * g.nz;
            // the in-place array (row blocks): lbm_create's limit, restated
            if ((19ll * g.pitch * g.nyp + 40ll * 32 * g.pitch + 2ll * g.pitch) * e < (1ll << 32))
                check(g, Layout{true, g.S, g.pitch, g.nyp, R}, e, false);
            // canonical arrays of the push and adjoint: eight slices with a
            // free-slip y or z face, else two, below 2^32 bytes
            bool freeslip = false;
            for (int k = 2; k < 6; k++) freeslip = freeslip || c.face[k] == 3;
            const long long span = freeslip ? 8 : 2;
            if (span * g.N * e < (1ll << 32)) {
                check(g, Layout{false, g.N, g.nx, g.ny, 1}, e, false);   // push
                check(g, Layout{false, g.N, g.nx, g.ny, 1}, e, true);    // adjoint
            }
        }
    }
    std::printf("checked %lld addresses, %lld errors\n", checked, errors);
    return errors ? 1 : 0;
}
'''


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_slot_offsets_resolve_inside_the_array(tmp_path):
    src = tmp_path / "offsets.hip"
    src.write_text(SRC)
    exe = tmp_path / "offsets"
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    # host code built with AddressSanitizer and UBSan (device code untouched)
    subprocess.check_call([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-I", INC, "-I", CSRC,
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=undefined", str(src), "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    assert "0 errors" in r.stdout


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbm.so not built")
def test_create_refuses_grids_beyond_32bit_offsets():
    """A grid whose in-place offsets would not fit 32 bits (19 populations
    of one xy plane reach 4 GiB) is refused before any device call or any read
    of the (here one-byte) solid mask."""
    from paper_2607_04516_amd import binding
    lib = binding.load()
    p = binding._Params()
    p.tau0, p.c_smag, p.delta, p.rho0 = 0.6, 0.1, 1.0, 1.0
    p.storage = binding.F32
    solid = (ctypes.c_uint8 * 1)()
    cases = [((8192, 8192, 3), (1, 2, 1, 2, 4, 4)),   # 19 populations of an xy plane: 5.1 GB in FP32
             ((16384, 4096, 3), (1, 2, 3, 3, 4, 3))]
    for dims, faces in cases:
        for k in range(6):
            p.face[k] = faces[k]
        ctx = ctypes.c_void_p()
        g = binding._Grid(*dims)
        rc = lib.lbm_create(ctypes.byref(g), ctypes.cast(solid, ctypes.c_void_p), ctypes.byref(p), ctypes.byref(ctx))
        assert rc == binding.LBM_EINVAL and not ctx.value, dims
        assert b"too large" in lib.lbm_last_error(None)
