// The two in-place A-A step kernels of the D3Q19 LBM-LES update on gfx950.
//
// Even step (natural layout -> swapped): every fluid cell reads its own 19
// slots, collides, and writes f*_i into its own slot opp(i).  No boundary
// rule is involved, so one kernel covers every wave.
//
// Odd step (swapped -> natural): the pull of direction I at cell x reads
// the slot (x - c_I, opp(I)) (or its boundary substitute) and the push of
// opp(I) writes back into the same slot.  This kernel takes every wave whose
// row is not on a y or z face; the remaining waves go to the general kernel
// through a wave list built at context creation.  Inside this kernel:
//   * one 32-bit lane offset addresses all 19 slots: each direction has its
//     own wave-uniform 64-bit base (slice base minus the neighbour offset);
//   * halfway bounce-back at solid neighbours is a per-lane select between
//     the neighbour slot and the cell's own slot, driven by 64-bit lane masks
//     that the scalar unit builds from the bit-packed solid rows (a row word
//     covers exactly the 64 lanes of a wave);
//   * the inflow cell of an x- INFLOW face (lane 0 of chunk 0) writes
//     feq(rho0, u_in), the outflow cell of an x+ OUTFLOW face reads its five
//     entering populations from the ghost plane.
#include "lbm_device.h"
#include "lbm_general.h"
#include "lbm_launch.h"

#include <type_traits>

namespace lbm {

template <int I, int N, class Fn>
__device__ __forceinline__ void sfor(Fn&& fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        sfor<I + 1, N>(fn);
    }
}

// Block order.  Blocks are dealt round robin to the 8 XCDs (hardware block
// i runs on XCD i % 8), each with its own L2.  The odd step's x-shifted
// pulls share the 128-byte lines at chunk edges with the neighbouring wave,
// so its grid places pairs of consecutive blocks (eight consecutive chunks)
// on one XCD: FP32 odd step 2.36 -> 2.34 ms on the kilometre grid, binary16
// unchanged; groups of four or eight blocks were slower.  The even step
// shares no lines and keeps the plain order.
constexpr long long XCD_GROUP = 2;
__device__ inline long long xcd_grouped_block()
{
    const long long i = blockIdx.x;
    const long long slot = i >> 3, xcd = i & 7;
    return (slot / XCD_GROUP) * (8 * XCD_GROUP) + xcd * XCD_GROUP + (slot % XCD_GROUP);
}

// Population traffic of the step kernels.  The even step touches each line
// once: with the row-block layout, non-temporal (streaming) loads and stores
// took the FP32 even step from 2.54 to 2.13 ms on the kilometre grid; 16-bit
// storage is fastest with non-temporal stores only (1.16 ms, against 1.20
// with both).  On the 256x256x96 adjoint grid (0.48 GB, twice the
// last-level cache) the hint still pays: the even step 196 -> 185 us, and
// the odd step that follows 188 -> 151 us.  The odd step's x-shifted pulls
// share the lines at chunk edges with the neighbouring waves and stay plain
// (the hint on every direction made the odd step 19% slower); its
// directions with c_x = 0 take it (ld_odd / st_odd).  The push recompute is
// slower with the hint on its loads (215 -> 229 us), on all its scattered
// stores (281 us) or on its stores with c_x = 0 (221 us).
template <typename T>
__device__ inline T ld_pop(const T* p)
{
    return *p;
}
template <typename T>
__device__ inline void st_pop(T* p, T v)
{
    *p = v;
}
template <typename T>
__device__ inline T ld_stream(const T* p)
{
    if constexpr (sizeof(T) >= 4) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename T>
__device__ inline void st_stream(T* p, T v)
{
    __builtin_nontemporal_store(v, p);
}
// Odd-step access of direction I: the slots of directions with c_x = 0 are
// read and written at the wave's own 64-cell x range (whole lines that no
// other wave touches) and take non-temporal hints at every storage width;
// the x-shifted ones share their chunk-edge lines with the neighbouring
// wave and stay plain.  On the 800x800x128 grid: FP32 odd 2509 -> 2356 us,
// binary16 1431 -> 1375 us (loads and stores both hinted; either alone, or
// stores hinted in every direction, is slower).
template <int I, typename T>
__device__ inline T ld_odd(const T* p)
{
    if constexpr (dirv(I).x == 0) return __builtin_nontemporal_load(p);
    else return *p;
}
template <int I, typename T>
__device__ inline void st_odd(T* p, T v)
{
    if constexpr (dirv(I).x == 0) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename R>
__device__ inline void inflow_eq_stored(const double* __restrict__ uin, const Geo& g, int face, int x, int y, int z,
                                        R rho0, R sc, R* h)
{
    const double* p = uin + 3 * inflow_slot(g, face, x, y, z);
    equilibrium_shifted<R>(rho0, R(0), R(p[0]), R(p[1]), R(p[2]), h);
#pragma unroll
    for (int i = 0; i < NQ; i++) h[i] *= sc;
}

template <typename R>
__device__ inline void add_stats(R* stats, const Geo& g, int x, int y, int z, R ux, R uy, R uz)
{
    const long long n = x + (long long)g.nx * (y + (long long)g.ny * z);
    stats[n] += ux;
    stats[g.N + n] += uy;
    stats[2 * g.N + n] += uz;
    stats[3 * g.N + n] += ux * ux;
    stats[4 * g.N + n] += uy * uy;
    stats[5 * g.N + n] += uz * uz;
}

// Probe sampling inside the step: a lane whose cell is a registered probe
// adds the velocity of the state the step starts from (the moments the
// collision formed, before any nudging) to each of its probes' Neumaier
// sums, in the arithmetic of the separate probe kernel.  Only waves whose
// chunk bit is set search the sorted table; a probe's sums are written by
// the one lane holding its cell.
__device__ inline bool step_chunk_has_probe(const StepProbes& pr, long long wave)
{
    return ((pr.bits[wave >> 5] >> (wave & 31)) & 1u) != 0;
}

template <typename R>
__device__ inline void step_probe_add(const StepProbes& pr, long long cell, long long cell0, R ux, R uy, R uz)
{
    int lo = 0, hi = pr.n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)pr.cell[mid] < cell0) lo = mid + 1;
        else hi = mid;
    }
    R* acc = (R*)pr.acc;
    auto add = [](R* sum, R* cmp, R xa) {
        const R sa = *sum;
        const R t = sa + xa;
        *cmp += fabs(sa) >= fabs(xa) ? (sa - t) + xa : (xa - t) + sa;
        *sum = t;
    };
    for (int e = lo; e < pr.n && (long long)pr.cell[e] < cell0 + 64; e++) {
        if ((long long)pr.cell[e] != cell) continue;
        const int p = pr.id[e];
        R* sum = acc + 3 * p;
        R* cmp = acc + 3 * (long long)pr.n + 3 * p;
        add(sum, cmp, ux);
        add(sum + 1, cmp + 1, uy);
        add(sum + 2, cmp + 2, uz);
    }
}

// ---------------------------------------------------------------- even step
// Occupancy is left to the compiler (seven waves per SIMD at FP32, its
// scalar registers): asking for eight, which made it spill scalar registers
// into vector lanes, was 2.3% slower on the kilometre grid and 2.9% on the
// 256x256x96 grid with the current streaming hints.
template <int K, bool STATS, bool PROBES>
__global__ void __launch_bounds__(256)
k_even(typename Codec<K>::store* f, const uint64_t* __restrict__ mask, const double* __restrict__ uin, Geo g,
       Phys<typename Codec<K>::real> P, StepOff O, typename Codec<K>::real* stats, StepProbes pr, long long nwaves,
       WaveDiv wd)
{
    using C = Codec<K>;
    using R = typename C::real;
    using T = typename C::store;
    const long long wave = (long long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int lane = threadIdx.x & 63;
    // (cx, y, z) of the wave by multiply-high divisions (nwaves < 2^32), a
    // dozen scalar instructions in place of two 64-bit divisions: binary16
    // step 1.316 -> 1.309 ms on the kilometre grid, FP32 unchanged
    const uint32_t r32 = fdiv((uint32_t)wave, wd.ncx), z32 = fdiv(r32, wd.ny);
    const int cx = (int)((uint32_t)wave - r32 * (uint32_t)g.ncx);
    const long long row = r32;
    const int y = (int)(r32 - z32 * (uint32_t)g.ny), z = (int)z32;
    const int x = cx * 64 + lane;
    const uint64_t wrow = mask_word(mask, row * g.wpr + cx);
    if (x >= g.nx || ((wrow >> lane) & 1ull)) return;

    char* base = (char*)f + row_start(g, mem_row(g, y, z), (int)sizeof(T));
    const uint32_t off = (uint32_t)x * (uint32_t)sizeof(T);
    R h[NQ];
    const int inf = inflow_face_of(g, x, y, z);
    if (inf >= 0) {
        inflow_eq_stored<R>(uin, g, inf, x, y, z, P.rho0, R(C::SC), h);
        if constexpr (STATS) {
            const double* p = uin + 3 * inflow_slot(g, inf, x, y, z);
            add_stats<R>(stats, g, x, y, z, R(p[0]), R(p[1]), R(p[2]));
        }
        sfor<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            st_stream((T*)(base + O.even[I] + off), C::pack(h[opp(I)]));
        });
        return;
    }
    sfor<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        h[I] = C::raw(ld_stream((const T*)(base + O.even[I] + off)));
    });
    R drho, ux, uy, uz, tau;
    collide_at<R, C::SC>(h, P, g, x, y, z, drho, ux, uy, uz, tau);
    sfor<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        st_stream((T*)(base + O.even[I] + off), C::pack(h[opp(I)]));
    });
    if constexpr (STATS) add_stats<R>(stats, g, x, y, z, ux, uy, uz);
    if constexpr (PROBES)
        if (step_chunk_has_probe(pr, wave)) step_probe_add<R>(pr, x + (long long)g.nx * row, (long long)g.nx * row + cx * 64, ux, uy, uz);
}

// Waves the odd kernel below leaves to the general kernel (same test on
// the host, see odd_wave_is_general in the runtime).
__device__ inline bool odd_general_wave(const Geo& g, int cx, int y, int z)
{
    return odd_wave_is_general(g, cx, y, z);
}

// ---------------------------------------------------------------- odd step
template <int K, bool STATS, bool PROBES>
__global__ void __launch_bounds__(256)
k_odd(typename Codec<K>::store* f, const uint64_t* __restrict__ mask, const int* __restrict__ wave_idx,
      const uint64_t* __restrict__ wave_tab, const double* __restrict__ uin,
      const typename Codec<K>::store* __restrict__ ghost, Geo g, Phys<typename Codec<K>::real> P,
      const StepOff* __restrict__ otab, typename Codec<K>::real* stats, StepProbes pr, long long nwaves, WaveDiv wd)
{
    using C = Codec<K>;
    using R = typename C::real;
    using T = typename C::store;
    // the grid is a multiple of 8 XCD_GROUP blocks, so the grouped order is a
    // permutation of the blocks
    const long long wave = xcd_grouped_block() * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int lane = threadIdx.x & 63;
    const uint32_t r32 = fdiv((uint32_t)wave, wd.ncx), z32 = fdiv(r32, wd.ny);
    const int cx = (int)((uint32_t)wave - r32 * (uint32_t)g.ncx);
    const long long row = r32;
    const int y = (int)(r32 - z32 * (uint32_t)g.ny), z = (int)z32;
    if (odd_general_wave(g, cx, y, z)) return;
    const int x = cx * 64 + lane;
    const auto& O = class_offsets(otab, 4 * row_class(g, y, z) + block_edge(g, mem_row(g, y, z)));
    const bool x_lo = (cx == 0);                   // lane 0 is an x- inflow or wall cell
    const bool x_hi = (cx * 64 + 63 >= g.nx - 1);  // lane l_out is an x+ outflow or wall cell
    const int l_out = (g.nx - 1) - cx * 64;

    // Solid-source masks: 16-bit storage leaves the kernel issue-bound, so it
    // reads them from the per-wave table (18 scalar loads, no mask
    // arithmetic); wider storage is bandwidth-bound and builds them from the
    // mask rows, whose words neighbouring waves share in the scalar cache
    // (the table entry is a cold load ahead of every wave's first access).
    constexpr bool ROWS = sizeof(T) >= 4;
    RowWin W;
    WaveMask WM{nullptr};
    uint64_t own;
    bool solid_any;
    if constexpr (ROWS) {
        load_rows(W, mask, g, cx, y, z);
        own = W.c[1][1];
        uint64_t a = 0;
        sfor<1, NQ>([&](auto ic) { a |= solid_src_mask<decltype(ic)::value>(W); });
        solid_any = uniform_u64(a) != 0;
    } else {
        WM = wave_mask(wave_idx, wave_tab, wave);
        own = mask_word(mask, row * g.wpr + cx);
        solid_any = WM.m != nullptr;
    }
    if (x >= g.nx || ((own >> lane) & 1ull)) return;

    // bounce mask of direction I: bit l set when lane l must use its own
    // slot (solid neighbour, or an x-face lane's face-crossing direction)
    auto bmask = [&](auto ic) -> uint64_t {
        constexpr int I = decltype(ic)::value;
        constexpr V3 c = dirv(I);
        uint64_t m;
        if constexpr (ROWS) m = solid_src_mask<I>(W);
        else m = WM.template get<I>();
        if constexpr (c.x == 1) { if (x_lo) m |= 1ull; }
        if constexpr (c.x == -1) { if (x_hi) m |= 1ull << l_out; }
        return m;
    };

    char* base = (char*)f + row_start(g, mem_row(g, y, z), (int)sizeof(T));
    const uint32_t off = (uint32_t)x * (uint32_t)sizeof(T);
    R h[NQ];
    if (!solid_any && !x_lo && !x_hi) {
        // fast path: no solid neighbour, no face lane
        sfor<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            h[I] = C::raw(ld_odd<I>((const T*)(base + O.odd[I] + off)));
        });
        R drho, ux, uy, uz, tau;
        collide_at<R, C::SC>(h, P, g, x, y, z, drho, ux, uy, uz, tau);
        sfor<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            st_odd<I>((T*)(base + O.odd[I] + off), C::pack(h[opp(I)]));
        });
        if constexpr (STATS) add_stats<R>(stats, g, x, y, z, ux, uy, uz);
        if constexpr (PROBES)
            if (step_chunk_has_probe(pr, wave)) step_probe_add<R>(pr, x + (long long)g.nx * row, (long long)g.nx * row + cx * 64, ux, uy, uz);
        return;
    }

    // masked path: per direction, slot = own (x, I) where the mask bit is set,
    // else (x - c_I, opp(I)); both addressed from the lower of the two slices
    uint32_t so[NQ];
    sfor<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if constexpr (I == 0) {
            so[0] = off;
        } else {
            so[I] = lane_select(off + O.on[I], off + O.oo[I], bmask(ic));
        }
    });
    sfor<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        h[I] = C::raw(ld_odd<I>((const T*)(base + O.lo[I] + so[I])));
    });
    const bool inflow_lane = x_lo && g.face[0] == F_INFLOW && lane == 0;
    const bool outflow_lane = x_hi && g.face[1] == F_OUTFLOW && lane == l_out;
    if (outflow_lane) {
        // entering populations of the x+ outflow cell: the ghost plane
        const long long fc = (long long)g.ny * g.nz;
        const long long gi = g.ghost_off[1] + y + (long long)g.ny * z;
        h[2] = C::raw(ghost[gi]);
        h[8] = C::raw(ghost[gi + fc]);
        h[10] = C::raw(ghost[gi + 2 * fc]);
        h[14] = C::raw(ghost[gi + 3 * fc]);
        h[16] = C::raw(ghost[gi + 4 * fc]);
    }
    R ux, uy, uz;
    if (inflow_lane) {
        inflow_eq_stored<R>(uin, g, 0, 0, y, z, P.rho0, R(C::SC), h);
        const double* p = uin + 3 * inflow_slot(g, 0, 0, y, z);
        ux = R(p[0]);
        uy = R(p[1]);
        uz = R(p[2]);
    } else {
        R drho, tau;
        collide_at<R, C::SC>(h, P, g, x, y, z, drho, ux, uy, uz, tau);
    }
    sfor<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        st_odd<I>((T*)(base + O.lo[I] + so[I]), C::pack(h[opp(I)]));
    });
    if constexpr (STATS) add_stats<R>(stats, g, x, y, z, ux, uy, uz);
    // (the runtime registers no x-face cell as a probe sampled here)
    if constexpr (PROBES)
        if (step_chunk_has_probe(pr, wave)) step_probe_add<R>(pr, x + (long long)g.nx * row, (long long)g.nx * row + cx * 64, ux, uy, uz);
}

// ---------------------------------------------------------------- push step
// Out-of-place step on canonical (unpadded) arrays, src -> dst, in one
// launch with two kinds of blocks, in the order of the context's block
// schedule.  Per-cell blocks run the general per-cell code for the face
// layer outside main_box(g, 0) (the listed cells); inflow cells among them
// write their canonical equilibrium into their own slots.  Wave blocks take
// the waves of main_box(g, 0), and with an inflow x- and an outflow x+ face
// also the x-face cells of the rows push_x_edge_row names:
// local read, collision, push of f*_opp(I) into the slot the pull of I
// resolves to (own slot at solid neighbours and across WALL faces).  Waves
// next to an INFLOW face skip the pushes that land in an inflow cell, so
// the two kinds of blocks write disjoint slots and run side by side, each
// per-cell block next to the wave blocks of its rows.  Solid cells get 0.
// The zero-gradient outflow copies are stored together with the slots they
// copy (no copy pass follows): on the backward workload's grid that removed
// a 12.7 us launch per step, the push itself unchanged at 201 us.

// Whether the push of f*_opp(I) from (x, y, z) lands in an inflow cell: the
// pull source x - c_I resolved through FREESLIP (mirror) and PERIODIC
// (wrap) faces lies on an INFLOW face layer.  Across a WALL face the value
// stays in the cell's own slot; a solid source does too, which the caller
// tests with the lane masks.  Cells of main_box(g, 0) never cross an
// INFLOW or OUTFLOW face.
// One axis of the resolution: the coordinate p = own - c of the pull
// source, mirrored or wrapped; false when the value stays in the own slot.
__device__ inline bool resolve_axis(int& p, int own, int n, int kind_lo, int kind_hi)
{
    if (p >= 0 && p < n) return true;
    const int kind = p < 0 ? kind_lo : kind_hi;
    if (kind == F_FREESLIP) p = own;
    else if (kind == F_PERIODIC) p = p < 0 ? n - 1 : 0;
    else return false;
    return true;
}

template <int I>
__device__ inline bool push_lands_in_inflow(const Geo& g, int x, int y, int z)
{
    constexpr V3 c = dirv(I);
    int px = x - c.x, py = y - c.y, pz = z - c.z;
    if constexpr (c.x != 0)
        if (!resolve_axis(px, x, g.nx, g.face[0], g.face[1])) return false;
    if constexpr (c.y != 0)
        if (!resolve_axis(py, y, g.ny, g.face[2], g.face[3])) return false;
    if constexpr (c.z != 0)
        if (!resolve_axis(pz, z, g.nz, g.face[4], g.face[5])) return false;
    return inflow_face_of(g, px, py, pz) >= 0;
}

template <int K>
__global__ void __launch_bounds__(256)
k_push(const typename Codec<K>::store* __restrict__ src, typename Codec<K>::store* __restrict__ dst,
       const uint64_t* __restrict__ mask, const int* __restrict__ wave_idx, const uint64_t* __restrict__ wave_tab,
       const double* __restrict__ uin, Geo g, Phys<typename Codec<K>::real> P, const StepOff* __restrict__ otab,
       long long nwaves, const unsigned* __restrict__ cells, long long ncells, const unsigned* __restrict__ sched)
{
    using C = Codec<K>;
    using R = typename C::real;
    using T = typename C::store;
    const unsigned code = sched[blockIdx.x];
    const unsigned idx = code & 0x3fffffffu;
    if ((code >> 30) == 0) {
        const long long t = idx * 256ll + threadIdx.x;
        if (t >= ncells) return;
        const long long n = cells[t];
        const long long r = n / g.nx;
        const Lay L{g.N, g.nx, -1, g.ny};
        general_cell<K, MODE_PUSH, false>(dst, src, mask, uin, nullptr, g, L, L, P, nullptr, (int)(n % g.nx),
                                          (int)(r % g.ny), (int)(r / g.ny));
        return;
    }
    const long long wave = idx * 4ll + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int lane = threadIdx.x & 63;
    const int cx = (int)(wave % g.ncx);
    const long long row = wave / g.ncx;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    const Box B = main_box(g, 0);
    if (y < B.y0 || y > B.y1 || z < B.z0 || z > B.z1) return;
    const int x = cx * 64 + lane;
    const auto& O = class_offsets(otab, row_class(g, y, z));
    // masks as in the odd kernel: cached mask rows for 32-bit and wider
    // storage, the per-wave table for 16-bit storage
    constexpr bool ROWS = sizeof(T) >= 4;
    RowWin W;
    WaveMask WM{nullptr};
    uint64_t own;
    bool solid_any;
    if constexpr (ROWS) {
        load_rows(W, mask, g, cx, y, z);
        own = W.c[1][1];
        uint64_t a = 0;
        sfor<1, NQ>([&](auto ic) { a |= solid_src_mask<decltype(ic)::value>(W); });
        solid_any = uniform_u64(a) != 0;
    } else {
        WM = wave_mask(wave_idx, wave_tab, wave);
        own = mask_word(mask, row * g.wpr + cx);
        solid_any = WM.m != nullptr;
    }
    auto smask = [&](auto ic) -> uint64_t {
        constexpr int I = decltype(ic)::value;
        if constexpr (ROWS) return solid_src_mask<I>(W);
        else return WM.template get<I>();
    };
    // rows whose x-face cells this wave takes as well (inflow x-, outflow x+)
    const bool xr = push_x_edge_row(g, ROWS, y, z);
    if (x >= g.nx || (!xr && (x < B.x0 || x > B.x1))) return;
    const uint32_t off = (uint32_t)((long long)x + (long long)g.nx * row) * (uint32_t)sizeof(T);
    const char* sbase = (const char*)src;
    char* dbase = (char*)dst;
    // lane masks (wave-uniform): the inflow cell x = 0, its neighbour x = 1,
    // the outflow face cell x = nx - 1
    const uint64_t e0 = (xr && cx == 0) ? 1ull : 0ull;
    const uint64_t e1 = (xr && cx == 0) ? 2ull : 0ull;
    const int la = g.nx - 1 - cx * 64;
    const uint64_t ea = (xr && la >= 0 && la < 64) ? 1ull << la : 0ull;
    // A solid lane writes 0 into its own 19 slots with the same store
    // instructions as the fluid lanes (no fluid lane pushes into a solid
    // cell, so the addresses never collide).
    const bool solid_lane = (own >> lane) & 1ull;
    R h[NQ];
    if (!solid_lane) {
        sfor<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            h[I] = C::raw(ld_pop((const T*)(sbase + O.even[I] + off)));
        });
    } else {
        sfor<0, NQ>([&](auto ic) { h[decltype(ic)::value] = R(0); });
    }
    R drho, ux, uy, uz, tau;
    collide_at<R, C::SC>(h, P, g, x, y, z, drho, ux, uy, uz, tau);
    // Zero-gradient outflow copies (the push stores them with the slots they
    // copy; no copy pass follows).  A wave-path cell writes a copied slot in
    // two ways only: a bounce-back into its own slot I when it lies next to
    // an outflow face I enters through (copied one cell outward, along each
    // such face and both at an edge), and, as the x+ face cell of a row
    // whose x-face cells the wave takes, a push of a direction with c_x = 1
    // into the cell at nx - 2 (copied back into the face cell of the row it
    // lands in, one element further along x).  Wave-uniform gate: the wave
    // holds a cell next to or on an outflow face.
    {
        const bool ox1 = g.face[1] == F_OUTFLOW, ox0 = g.face[0] == F_OUTFLOW;
        const bool nyp = g.face[3] == F_OUTFLOW && y == g.ny - 2, nym = g.face[2] == F_OUTFLOW && y == 1;
        const bool nzp = g.face[5] == F_OUTFLOW && z == g.nz - 2, nzm = g.face[4] == F_OUTFLOW && z == 1;
        const bool wx = (ox1 && cx * 64 + 63 >= g.nx - 2) || (ox0 && cx == 0);
        if (wx || nyp || nym || nzp || nzm) {
            const bool fluid_lane = !solid_lane && inflow_face_of(g, x, y, z) < 0;
            const bool nxp = ox1 && x == g.nx - 2, nxm = ox0 && x == 1;
            const bool face_lane = fluid_lane && xr && ox1 && x == g.nx - 1;
            const Lay L{g.N, g.nx, -1, g.ny};
            sfor<1, NQ>([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                constexpr V3 c = dirv(I);
                const bool bb = ((smask(ic) >> lane) & 1ull) != 0;
                const int sx = (c.x == -1 && nxp) ? 1 : ((c.x == 1 && nxm) ? -1 : 0);
                const int sy = (c.y == -1 && nyp) ? 1 : ((c.y == 1 && nym) ? -1 : 0);
                const int sz = (c.z == -1 && nzp) ? 1 : ((c.z == 1 && nzm) ? -1 : 0);
                if (fluid_lane && bb && (sx | sy | sz) != 0) {
                    for (int sub = 1; sub < 8; sub++) {
                        if (((sub & 1) && !sx) || ((sub & 2) && !sy) || ((sub & 4) && !sz)) continue;
                        const int tx = x + ((sub & 1) ? sx : 0);
                        const int ty = y + ((sub & 2) ? sy : 0);
                        const int tz = z + ((sub & 4) ? sz : 0);
                        if (!solid_at(mask, g, tx, ty, tz) && inflow_face_of(g, tx, ty, tz) < 0)
                            dst[pop_index(L, I, tx, ty, tz)] = C::pack(h[opp(I)]);
                    }
                }
                if constexpr (c.x == 1) {
                    // the row the push lands in holds fluid at x = nx - 1
                    // (the mask window mirrors rows at free-slip faces)
                    constexpr int KT = dir_index(0, c.y, c.z);
                    bool tsolid = false;
                    if constexpr (KT != 0) tsolid = ((smask(std::integral_constant<int, KT>{}) >> lane) & 1ull) != 0;
                    if (face_lane && !bb && !tsolid)
                        st_pop((T*)(dbase + O.lo[I] + (off + O.on[I] + (uint32_t)sizeof(T))), C::pack(h[opp(I)]));
                }
            });
        }
    }
    if ((e0 | e1 | ea) != 0) {
        // x-face cells of the row.  The inflow cell x = 0 outputs its own
        // equilibrium in its own slots and pushes it toward x = 1; the
        // populations of x = 1 moving to x = 0 are dropped (unless x = 0 is
        // solid: bounce-back); those of the outflow face cell leaving through
        // the face are dropped unless the cell at nx - 2 is solid (then they
        // are its bounce-back).
        if (e0 != 0 && !solid_lane && lane == 0) {
            R vx, vy, vz, heq[NQ];
            load_inflow<R>(uin, g, 0, 0, y, z, vx, vy, vz);
            equilibrium_shifted<R>(P.rho0, R(0), vx, vy, vz, heq);
#pragma unroll
            for (int i = 0; i < NQ; i++) h[i] = heq[i] * R(C::SC);
        }
        const uint64_t xm_solid = smask(std::integral_constant<int, 1>{});   // cell x - 1 of the row is solid
        const bool inflow_lane = ((e0 >> lane) & 1ull) != 0;
        sfor<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            constexpr V3 c = dirv(I);
            if constexpr (I == 0) {
                st_pop((T*)(dbase + off), C::pack(solid_lane ? R(0) : h[0]));
            } else {
                const uint64_t sm = smask(ic);
                uint64_t force = own | e0;
                uint64_t skip = 0;
                if constexpr (c.x == 1) skip = e1 & ~sm & ~own;
                if constexpr (c.x == -1) {
                    force |= ea;
                    skip = ea & ~xm_solid & ~own;
                }
                const uint32_t so = lane_select(off + O.on[I], off + O.oo[I], sm | force);
                const R v = solid_lane ? R(0) : (inflow_lane ? h[I] : h[opp(I)]);
                if (!((skip >> lane) & 1ull)) st_pop((T*)(dbase + O.lo[I] + so), C::pack(v));
                if constexpr (c.x == -1) {
                    // off + on wraps modulo 2^32 like the other slot offsets
                    const uint32_t sn = off + O.on[I];
                    if (inflow_lane && !solid_lane && !(sm & 1ull)) st_pop((T*)(dbase + O.lo[I] + sn), C::pack(h[opp(I)]));
                }
            }
        });
        return;
    }
    // INFLOW face layers next to this wave (wave-uniform): the x- layer
    // when the chunk holds x = 1, the x+ layer when it holds x = nx - 2, the
    // y and z layers when the row is next to them.  Only a direction whose
    // pull source moves toward such a layer can land in an inflow cell.
    const int x0 = cx * 64;
    const bool in_x0 = g.face[0] == F_INFLOW && x0 <= 1, in_x1 = g.face[1] == F_INFLOW && x0 + 63 >= g.nx - 2;
    const bool in_y0 = g.face[2] == F_INFLOW && y == 1, in_y1 = g.face[3] == F_INFLOW && y == g.ny - 2;
    const bool in_z0 = g.face[4] == F_INFLOW && z == 1, in_z1 = g.face[5] == F_INFLOW && z == g.nz - 2;
    if (in_x0 || in_x1 || in_y0 || in_y1 || in_z0 || in_z1) {
        sfor<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            constexpr V3 c = dirv(I);
            if constexpr (I == 0) {
                st_pop((T*)(dbase + off), C::pack(solid_lane ? R(0) : h[0]));
            } else {
                const bool sol = solid_lane || (solid_any && ((smask(ic) >> lane) & 1ull));
                const bool toward = (c.x == 1 && in_x0) || (c.x == -1 && in_x1) || (c.y == 1 && in_y0) ||
                                    (c.y == -1 && in_y1) || (c.z == 1 && in_z0) || (c.z == -1 && in_z1);
                if (toward && !sol && push_lands_in_inflow<I>(g, x, y, z)) return;
                const uint32_t so = sol ? off + O.oo[I] : off + O.on[I];
                st_pop((T*)(dbase + O.lo[I] + so), C::pack(solid_lane ? R(0) : h[opp(I)]));
            }
        });
        return;
    }
    if (!solid_any) {   // then no lane is solid either
        sfor<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            st_pop((T*)(dbase + O.odd[I] + off), C::pack(h[opp(I)]));
        });
        return;
    }
    sfor<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if constexpr (I == 0) {
            st_pop((T*)(dbase + off), C::pack(solid_lane ? R(0) : h[0]));
        } else {
            const uint32_t so = lane_select(off + O.on[I], off + O.oo[I], smask(ic) | own);
            st_pop((T*)(dbase + O.lo[I] + so), C::pack(solid_lane ? R(0) : h[opp(I)]));
        }
    });
}


template <int K, bool STATS, bool PROBES>
static hipError_t launch_fused_k(const DevCtx& d, int odd, void* stats, const StepProbes& pr, hipStream_t s)
{
    using C = Codec<K>;
    using R = typename C::real;
    const long long nwaves = (long long)d.g.ncx * d.g.ny * d.g.nz;
    const long long nb = (nwaves + 3) / 4;
    const Phys<R> P = phys_of<K>(d);
    auto* f = (typename C::store*)d.f;
    const WaveDiv wd{fast_div((uint32_t)d.g.ncx), fast_div((uint32_t)d.g.ny)};
    if (!odd) {
        const StepOff O = step_offsets_blocked(d.g.pitch, d.g.nyp, d.g.lrb, (int)sizeof(typename C::store), 0, 0);
        hipLaunchKernelGGL((k_even<K, STATS, PROBES>), dim3((unsigned)nb), dim3(256), 0, s, f, d.mask, d.uin, d.g, P,
                           O, (R*)stats, pr, nwaves, wd);
        return hipGetLastError();
    }
    const long long nbg = (nb + 8 * XCD_GROUP - 1) / (8 * XCD_GROUP) * (8 * XCD_GROUP);
    hipLaunchKernelGGL((k_odd<K, STATS, PROBES>), dim3((unsigned)nbg), dim3(256), 0, s, f, d.mask, d.wave_idx,
                       d.wave_tab, d.uin, (const typename C::store*)d.ghost, d.g, P, d.off_odd, (R*)stats, pr, nwaves,
                       wd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_general_odd(d, stats, s);
}

template <int K>
static hipError_t launch_fused(const DevCtx& d, int odd, void* stats, void* probe_acc, hipStream_t s)
{
    if (stats && probe_acc) return hipErrorInvalidValue;
    const StepProbes pr{d.probes.bits, d.probes.cell, d.probes.id, d.probes.n, probe_acc};
    if (probe_acc) return pr.n > 0 ? launch_fused_k<K, false, true>(d, odd, stats, pr, s) : hipErrorInvalidValue;
    if (stats) return launch_fused_k<K, true, false>(d, odd, stats, pr, s);
    return launch_fused_k<K, false, false>(d, odd, stats, pr, s);
}

template <int K>
static hipError_t launch_push_k(const DevCtx& d, const void* src, void* dst, hipStream_t s)
{
    using C = Codec<K>;
    const long long nwaves = (long long)d.g.ncx * d.g.ny * d.g.nz;
    hipLaunchKernelGGL((k_push<K>), dim3(d.push_sched_n), dim3(256), 0, s, (const typename C::store*)src,
                       (typename C::store*)dst, d.mask, d.wave_idx, d.wave_tab, d.uin, d.g, phys_of<K>(d), d.off_push,
                       nwaves, d.push_list, d.push_list_n, d.push_sched);
    return hipGetLastError();
}

hipError_t launch_push(const DevCtx& d, const void* src, void* dst, hipStream_t s)
{
    switch (d.codec) {
        case 0: return launch_push_k<0>(d, src, dst, s);
        case 1: return launch_push_k<1>(d, src, dst, s);
        case 2: return launch_push_k<2>(d, src, dst, s);
        case 3: return launch_push_k<3>(d, src, dst, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(const DevCtx& d, int odd, void* stats, void* probe_acc, hipStream_t s)
{
    switch (d.codec) {
        case 0: return launch_fused<0>(d, odd, stats, probe_acc, s);
        case 1: return launch_fused<1>(d, odd, stats, probe_acc, s);
        case 2: return launch_fused<2>(d, odd, stats, probe_acc, s);
        case 3: return launch_fused<3>(d, odd, stats, probe_acc, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
