// Internal interface between the C-ABI runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "lbm.h"
#include "lbm_device.h"

namespace lbm {

struct StepOff;

// Probe table of the adjoint step: (cell, probe) entries sorted by canonical
// cell index (probe order within a cell) and one bit per 64-cell chunk of a
// row (chunk cx + ncx * row) that holds a probe cell.
struct AdjProbes {
    const uint32_t* bits;
    const unsigned* cell;
    const int* id;
    int n;              // entries; 0: no probes
    const void* src;    // per call: [np][3] dL/du at the probes, or nullptr
};

// The same table for the forward step kernels, which add u of the state a
// step starts from to the probes' compensated sums acc [2][np][3] (real
// type of the codec).
// Division of a 32-bit n by a run-time invariant divisor d (1 <= d < 2^32)
// as a multiply-high and two shifts whose constants the host fixes once
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, Fig. 4.1): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1 (which fits 32 bits), t = hi32(m n) and
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0).
struct FastDiv {
    uint32_t m, s1, s2;
};

inline FastDiv fast_div(uint32_t d)
{
    int l = 0;
    while ((1ull << l) < d) l++;
    const uint64_t m = ((((1ull << l) - d) << 32) / d) + 1;
    return FastDiv{(uint32_t)m, (uint32_t)(l < 1 ? l : 1), (uint32_t)(l > 1 ? l - 1 : 0)};
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    const uint32_t t = (uint32_t)(((uint64_t)f.m * n) >> 32);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// The divisors of the step kernels' wave index: chunks per row, rows per
// z plane.
struct WaveDiv {
    FastDiv ncx, ny;
};

struct StepProbes {
    const uint32_t* bits;
    const unsigned* cell;
    const int* id;
    int n;
    void* acc;
};

// Everything a kernel launch needs to know about one context.
struct DevCtx {
    Geo g;
    int codec;            // 0 F64, 1 F32, 2 F16S, 3 BF16S
    void* f;              // in-place population array [19][nz][ny][pitch]
    const uint64_t* mask; // solid bits [nz][ny][wpr]
    void* ghost;          // outflow ghost entries
    const double* ubase;  // per-cell boundary states of the INFLOW_EQ faces (inflow_slot): sponge targets
    const double* uin;    // per-cell inflow velocities (inflow_slot); what the step kernels read
    const unsigned* odd_list;  // waves of the odd step left to the general kernel
    long long odd_list_n;
    const unsigned* push_list; // canonical indices of the face-layer cells the push's waves do not take
    long long push_list_n;
    const unsigned* adj_list;  // canonical indices of the face-shell cells the adjoint's waves do not take
    long long adj_list_n;
    const unsigned* push_sched;  // block order of the push launch (kind << 30 | index)
    unsigned push_sched_n;
    const unsigned* adj_sched;   // block order of the adjoint launch
    unsigned adj_sched_n;
    const int* wave_idx;       // per wave (chunk, row): entry in wave_tab, -1 without solid neighbour
    const uint64_t* wave_tab;  // [entries][18] solid-source masks
    const StepOff* off_odd;    // [9 row classes][4 block edges] offsets of the in-place array, store elements
    const StepOff* off_push;   // [9] canonical layout, store elements
    const StepOff* off_adj;    // [9] canonical layout, real (adjoint) elements
    double tau0, c_smag, delta, rho0, force[3];
    double omega[3];      // rotation vector in lattice units (Coriolis); zero: none
    int sponge_w;         // sponge / buffer layer width; 0: off
    double sponge_s;      // its strength s_max
    AdjProbes probes;     // registered probes (src unset)
    int lds_per_cu;       // bytes of LDS per compute unit (0: unknown)
};

// Collision parameters of a context in the codec's arithmetic type.
template <int K>
static inline Phys<typename Codec<K>::real> phys_of(const DevCtx& d)
{
    using R = typename Codec<K>::real;
    Phys<R> P;
    P.tau0 = R(d.tau0);
    P.ksmag = R(18.0 * (d.c_smag * d.delta) * (d.c_smag * d.delta));
    P.rho0 = R(d.rho0);
    for (int a = 0; a < 3; a++) {
        P.F[a] = R(d.force[a]);
        P.W2[a] = R(2.0 * d.omega[a]);
    }
    P.has_rot = (d.omega[0] != 0.0 || d.omega[1] != 0.0 || d.omega[2] != 0.0) ? 1 : 0;
    P.has_force = (P.has_rot || d.force[0] != 0.0 || d.force[1] != 0.0 || d.force[2] != 0.0) ? 1 : 0;
    P.sponge_w = d.sponge_s > 0.0 ? d.sponge_w : 0;
    P.sponge_s = R(d.sponge_s);
    P.target = d.ubase;
    return P;
}

// Byte offsets of the population slots a wave touches, fixed per grid,
// codec and row class, computed on the host (otherwise every wave rebuilds
// them with 64-bit scalar arithmetic).  Slice stride sb = S (padded in-place
// layout) or N (canonical layout) times the element size; the pull of
// direction I reads slot opp(I') of the source cell x - c', where I' and c'
// are I and c_I with the components mirrored at FREESLIP faces (row_class)
// flipped and zeroed; d_I is the element offset of x - c'.
struct StepOff {
    long long even[NQ];  // I sb: slot I of the own cell
    long long odd[NQ];   // opp(I') sb - d_I: the pull source of direction I
    long long lo[NQ];    // min(I, opp(I')) sb
    uint32_t on[NQ];     // (opp(I') - lo) sb - d_I, relative to lo (mod 2^32)
    uint32_t oo[NQ];     // (I - lo) sb: the own slot (bounce-back)
};

static inline StepOff step_offsets(long long slice, long long rowlen, long long ny, int elem, int cls = 0)
{
    StepOff o;
    const long long sb = slice * (long long)elem;
    const int my = cls / 3, mz = cls % 3;
    for (int i = 0; i < NQ; i++) {
        const V3 c = dirv(i);
        int m = 0;
        if ((my == 1 && c.y == 1) || (my == 2 && c.y == -1)) m |= 2;
        if ((mz == 1 && c.z == 1) || (mz == 2 && c.z == -1)) m |= 4;
        const int slot = opp(mirrored(i, m));
        const int lo = i < slot ? i : slot;
        const long long d =
            ((long long)c.x + rowlen * ((m & 2 ? 0 : c.y) + ny * (m & 4 ? 0 : c.z))) * (long long)elem;
        o.even[i] = i * sb;
        o.odd[i] = slot * sb - d;
        o.lo[i] = lo * sb;
        o.on[i] = (uint32_t)((slot - lo) * sb - d);
        o.oo[i] = (uint32_t)((i - lo) * sb);
    }
    return o;
}

// Slices spanned by the two candidate slots of one direction (own slot I and
// pull-source slot opp(I')), plus one for the lane offset inside a slice: 2
// when every row class is plain (opp(I) is next to I), 8 when a y or z face
// is FREESLIP (the remapped directions of its face rows reach up to seven
// slices away, e.g. 7 -> 14 in the y = 0 row).  The 32-bit slot offsets need
// span * (slice bytes) < 2^32.
__host__ __device__ inline long long slot_span(const int face[6])
{
    for (int k = 2; k < 6; k++)
        if (face[k] == F_FREESLIP) return 8;
    return 2;
}

// Rows per block of the in-place array, R = 2^lrb <= 32: the largest R for
// which rounding ny up to whole blocks adds at most ny / 16 padding rows;
// nyp = ny rounded up to a multiple of R (rows per z plane in memory).
static inline void row_blocks(int ny, int& lrb, int& nyp)
{
    for (lrb = 5; lrb > 0; lrb--) {
        const long long R = 1ll << lrb;
        if (((ny + R - 1) / R * R - ny) * 16 <= ny) break;
    }
    nyp = (int)((ny + (1ll << lrb) - 1) >> lrb << lrb);
}

// Element offset of slot s of the cell (x + dx, row + dy + nyp dz) from slot
// 0 of (x, row) in the row-block layout of the in-place array (R = 2^lrb
// rows per block, R dividing nyp, |dy| <= 1).  A neighbour in z is nyp / R
// blocks away; a neighbour in y lies in the same block unless the row is the
// first (edge bit 0, dy = -1) or last (edge bit 1, dy = +1) of its block,
// where the step into the adjacent block adds -/+ 18 B (B = R pitch).
static inline long long block_rel(long long pitch, long long nyp, int lrb, int s, int dx, int dy, int dz, int edge)
{
    const long long R = 1ll << lrb, B = R * pitch;
    long long o = s * B + dx + pitch * dy + (nyp / R) * dz * NQ * B;
    if (dy == -1 && (edge & 1)) o -= (NQ - 1) * B;
    if (dy == 1 && (edge & 2)) o += (NQ - 1) * B;
    return o;
}

// StepOff of the in-place array (row blocks) for row class cls and block
// edge: offsets from the cell's row start (slot 0 of x = 0) in bytes; the
// kernels add the row start to the base and x * elem as the lane offset, so
// lo + (x elem + on) (pull source) and lo + (x elem + oo) (own slot) are
// exact while on, oo + pitch elem < 2^32 (checked by lbm_create).
static inline StepOff step_offsets_blocked(long long pitch, long long nyp, int lrb, int elem, int cls, int edge)
{
    StepOff o;
    const int my = cls / 3, mz = cls % 3;
    for (int i = 0; i < NQ; i++) {
        const V3 c = dirv(i);
        int m = 0;
        if ((my == 1 && c.y == 1) || (my == 2 && c.y == -1)) m |= 2;
        if ((mz == 1 && c.z == 1) || (mz == 2 && c.z == -1)) m |= 4;
        const int slot = opp(mirrored(i, m));
        const long long own = block_rel(pitch, nyp, lrb, i, 0, 0, 0, edge) * elem;
        const long long nb =
            block_rel(pitch, nyp, lrb, slot, -c.x, (m & 2) ? 0 : -c.y, (m & 4) ? 0 : -c.z, edge) * elem;
        const long long lo = own < nb ? own : nb;
        o.even[i] = own;
        o.odd[i] = nb;
        o.lo[i] = lo;
        o.on[i] = (uint32_t)(nb - lo);
        o.oo[i] = (uint32_t)(own - lo);
    }
    return o;
}

// Row of (y, z) in the in-place array (y + nyp z).
__host__ __device__ inline long long mem_row(const Geo& g, int y, int z)
{
    return (long long)y + (long long)g.nyp * z;
}

// Byte offset of the start of memory row `row` (slot 0, x = 0) of the
// in-place array.
__host__ __device__ inline long long row_start(const Geo& g, long long row, int elem)
{
    const long long rmask = (1ll << g.lrb) - 1;
    return ((row >> g.lrb) * NQ * (rmask + 1) + (row & rmask)) * (long long)g.pitch * elem;
}

// Block-edge flags of a memory row (bit 0: first row of its block, bit 1: last).
__host__ __device__ inline int block_edge(const Geo& g, long long row)
{
    const long long rr = row & ((1ll << g.lrb) - 1);
    return (rr == 0 ? 1 : 0) | (rr == (1ll << g.lrb) - 1 ? 2 : 0);
}

typedef const StepOff __attribute__((address_space(4))) const_stepoff;

// The offsets of one row class from a per-context table of nine.
__device__ inline const const_stepoff& class_offsets(const StepOff* tab, int cls)
{
    return ((const const_stepoff*)tab)[cls];
}

// Host copy of the odd kernel's test for waves it leaves to the general
// kernel (k_odd in lbm_step.hip applies the same test).
// Rows on a y or z face other than WALL or FREESLIP, and chunks holding an
// x-face cell unless the x- face is INFLOW or WALL and the x+ face OUTFLOW
// or WALL.
__host__ __device__ inline bool odd_wave_is_general(const Geo& g, int cx, int y, int z)
{
    auto folded = [](int kind) { return kind == F_WALL || kind == F_FREESLIP; };
    if ((y == 0 && !folded(g.face[2])) || (y == g.ny - 1 && !folded(g.face[3]))) return true;
    if ((z == 0 && !folded(g.face[4])) || (z == g.nz - 1 && !folded(g.face[5]))) return true;
    if (cx == 0 && g.face[0] != F_INFLOW && g.face[0] != F_WALL) return true;
    if (cx * 64 + 63 >= g.nx - 1 && g.face[1] != F_OUTFLOW && g.face[1] != F_WALL) return true;
    return false;
}

// probe_acc: NULL, or the accumulator the step kernels add the probe
// velocities of the state at the step's start to (not together with stats).
hipError_t launch_step(const DevCtx& d, int odd, void* stats, void* probe_acc, hipStream_t s);
hipError_t launch_general_odd(const DevCtx& d, void* stats, hipStream_t s);
hipError_t launch_push(const DevCtx& d, const void* src, void* dst, hipStream_t s);
hipError_t launch_outflow_ghost(const DevCtx& d, hipStream_t s);
hipError_t launch_outflow_copy(const DevCtx& d, void* arr, int canonical_layout, hipStream_t s);
hipError_t launch_init(const DevCtx& d, const double* u0_dev, double amp, uint64_t seed, hipStream_t s);
hipError_t launch_export(const DevCtx& d, int phase, void* dst, hipStream_t s);
hipError_t launch_import(const DevCtx& d, const void* src, hipStream_t s);
hipError_t launch_macros(const DevCtx& d, int phase, void* rho, void* u, void* nut, hipStream_t s);
hipError_t launch_probe_points(const DevCtx& d, int phase, const float* pts, int np, float* out, hipStream_t s);
hipError_t launch_probe_cells(const DevCtx& d, int phase, const int* cells, int np, void* acc, hipStream_t s);
int mass_blocks(const Geo& g);
hipError_t launch_mass(const DevCtx& d, int phase, double* partial, double* out5, hipStream_t s);
// Net outward flux over the boundary cells (slot, face) of uin into phi_out[0]
// (device); with apply, also the uniform normal shift that zeroes it.
hipError_t launch_flux_balance(const int* slot, const int* face, long long n, double* uin, double* partial,
                               double* phi_out, int apply, hipStream_t s);
int flux_partial_count();
// Wave-mask table: pass 0 writes a 0/1 flag per wave into idx (solid
// neighbour or not); pass 1 fills tab for the waves whose idx >= 0.
hipError_t launch_wave_masks(const DevCtx& d, int* idx, uint64_t* tab, int pass, hipStream_t s);
// Ray-parity voxelizer (lbm_voxel.hip): OR the voxelized meshes into solid
// (host [nz][ny][nx]); err holds the message on failure.
int voxelize(const lbm_grid* grid, const double* tri, int32_t nt, const int32_t* starts, int32_t nm, int32_t passes,
             uint8_t* solid, std::string& err);

// Halo exchange of a slab along y: pack (unpack = 0) or unpack (1) the five
// crossing populations of side 0 (y-) or 1 (y+) at the context's phase.
hipError_t launch_halo(const DevCtx& d, int side, int phase, int unpack, void* buf, hipStream_t s);

hipError_t launch_adjoint(const DevCtx& d, const void* f_t, const void* lam_next, void* lam, const void* probe_src,
                          void* g_inflow, hipStream_t s);

}  // namespace lbm
