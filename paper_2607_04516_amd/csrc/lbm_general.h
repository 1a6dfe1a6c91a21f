// The general per-cell path of the collide-and-stream step: every boundary
// rule, one cell per lane.  Shared by the step kernels (lbm_kernels.hip) and
// the push kernel, which runs it for its face layer in the same launch.
#pragma once

#include "lbm_device.h"

#include <type_traits>

namespace lbm {

template <int I, int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1, N>(fn);
    }
}

constexpr int MODE_EVEN = 0, MODE_ODD = 1, MODE_PUSH = 2;

// The zero-gradient outflow copies of slot (d, J) in the push's output
// (J with velocity (vx, vy, vz)): f_J(c) = f_J(q) for an outflow cell c,
// fluid and not an inflow cell, where q is c moved one cell inward along
// every outflow face c lies on and J enters through.  The c whose q is d
// are d moved outward along a non-empty subset of the axes where d lies
// next to an outflow face J enters through (up to three: J has at most two
// non-zero components), provided d itself lies on no outflow face J enters
// through (else q(c) would move along that axis too).  The push stores
// these copies together with the slot, so no copy pass follows it.
template <typename T>
__device__ __forceinline__ void store_copies(T* dst, const uint64_t* __restrict__ mask, const Geo& g, const Lay& L,
                                             int dx, int dy, int dz, int J, int vx, int vy, int vz, T v)
{
    int sx = 0, sy = 0, sz = 0;
    if (vx == -1 && g.face[1] == F_OUTFLOW) { if (dx == g.nx - 1) return; if (dx == g.nx - 2) sx = 1; }
    if (vx == 1 && g.face[0] == F_OUTFLOW) { if (dx == 0) return; if (dx == 1) sx = -1; }
    if (vy == -1 && g.face[3] == F_OUTFLOW) { if (dy == g.ny - 1) return; if (dy == g.ny - 2) sy = 1; }
    if (vy == 1 && g.face[2] == F_OUTFLOW) { if (dy == 0) return; if (dy == 1) sy = -1; }
    if (vz == -1 && g.face[5] == F_OUTFLOW) { if (dz == g.nz - 1) return; if (dz == g.nz - 2) sz = 1; }
    if (vz == 1 && g.face[4] == F_OUTFLOW) { if (dz == 0) return; if (dz == 1) sz = -1; }
    if ((sx | sy | sz) == 0) return;
    for (int sub = 1; sub < 8; sub++) {
        if (((sub & 1) && !sx) || ((sub & 2) && !sy) || ((sub & 4) && !sz)) continue;
        const int cx = dx + ((sub & 1) ? sx : 0);
        const int cy = dy + ((sub & 2) ? sy : 0);
        const int cz = dz + ((sub & 4) ? sz : 0);
        if (!solid_at(mask, g, cx, cy, cz) && inflow_face_of(g, cx, cy, cz) < 0) dst[pop_index(L, J, cx, cy, cz)] = v;
    }
}

// Every boundary rule, per cell: the step of one cell (x, y, z) in any mode.
template <int K, int MODE, bool STATS>
__device__ inline void general_cell(typename Codec<K>::store* dst, const typename Codec<K>::store* src,
                                    const uint64_t* __restrict__ mask, const double* __restrict__ uin,
                                    const typename Codec<K>::store* __restrict__ ghost, const Geo& g, const Lay& ls,
                                    const Lay& ld, const Phys<typename Codec<K>::real>& P,
                                    typename Codec<K>::real* stats, int x, int y, int z)
{
    using C = Codec<K>;
    using R = typename C::real;
    if (solid_at(mask, g, x, y, z)) {
        if constexpr (MODE == MODE_PUSH) {
            static_for<0, NQ>([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                dst[pop_index(ld, I, x, y, z)] = C::enc(R(0));
            });
        }
        return;
    }
    R h[NQ];
    R ux, uy, uz;
    const int inf = inflow_face_of(g, x, y, z);
    if (inf >= 0) {
        // inflow cell: post-collision state is feq(rho0, u_in(z)) whatever it held
        load_inflow<R>(uin, g, inf, x, y, z, ux, uy, uz);
        equilibrium_shifted<R>(P.rho0, R(0), ux, uy, uz, h);
#pragma unroll
        for (int i = 0; i < NQ; i++) h[i] *= R(C::SC);
        static_for<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            if constexpr (MODE == MODE_EVEN) {
                dst[pop_index(ld, I, x, y, z)] = C::pack(h[opp(I)]);
            } else if constexpr (MODE == MODE_PUSH) {
                // canonical output of an inflow cell is its own equilibrium
                dst[pop_index(ld, I, x, y, z)] = C::pack(h[I]);
                const Res r = resolve_plain<I>(g, mask, x, y, z);
                if (r.kind == 0 && !(r.x == x && r.y == y && r.z == z) && inflow_face_of(g, r.x, r.y, r.z) < 0) {
                    dst[pop_index(ld, r.dir, r.x, r.y, r.z)] = C::pack(h[opp(I)]);
                    store_copies(dst, mask, g, ld, r.x, r.y, r.z, r.dir, r.vx, r.vy, r.vz, C::pack(h[opp(I)]));
                }
            } else {
                const Res r = resolve_plain<I>(g, mask, x, y, z);
                if (r.kind == 0)
                    dst[pop_index(ld, r.dir, r.x, r.y, r.z)] = C::pack(h[opp(I)]);
            }
        });
    } else {
        // gather
        static_for<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            if constexpr (MODE == MODE_ODD) {
                int qx, qy, qz, owner;
                if (outflow_entering<I>(g, x, y, z, qx, qy, qz, owner)) {
                    h[I] = C::raw(ghost[ghost_index<I>(g, owner, x, y, z)]);
                } else {
                    const Res r = resolve_plain<I>(g, mask, x, y, z);
                    h[I] = C::raw(src[pop_index(ls, r.dir, r.x, r.y, r.z)]);
                }
            } else {
                h[I] = C::raw(src[pop_index(ls, I, x, y, z)]);
            }
        });
        R drho, tau;
        collide_at<R, C::SC>(h, P, g, x, y, z, drho, ux, uy, uz, tau);
        // scatter
        static_for<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            if constexpr (MODE == MODE_EVEN) {
                dst[pop_index(ld, I, x, y, z)] = C::pack(h[opp(I)]);
            } else {
                int qx, qy, qz, owner;
                if (outflow_entering<I>(g, x, y, z, qx, qy, qz, owner)) {
                    // opp(I) leaves through the outflow face: kept only as the
                    // bounce-back of a solid inner neighbour
                    if (solid_at(mask, g, qx, qy, qz)) dst[pop_index(ld, I, x, y, z)] = C::pack(h[opp(I)]);
                } else {
                    const Res r = resolve_plain<I>(g, mask, x, y, z);
                    if (r.kind == 0) {
                        if constexpr (MODE == MODE_PUSH) {
                            if (inflow_face_of(g, r.x, r.y, r.z) >= 0) return;
                        }
                        dst[pop_index(ld, r.dir, r.x, r.y, r.z)] = C::pack(h[opp(I)]);
                        if constexpr (MODE == MODE_PUSH)
                            store_copies(dst, mask, g, ld, r.x, r.y, r.z, r.dir, r.vx, r.vy, r.vz, C::pack(h[opp(I)]));
                    }
                }
            }
        });
    }
    if constexpr (STATS) {
        const long long n = x + (long long)g.nx * (y + (long long)g.ny * z);
        stats[n] += ux;
        stats[g.N + n] += uy;
        stats[2 * g.N + n] += uz;
        stats[3 * g.N + n] += ux * ux;
        stats[4 * g.N + n] += uy * uy;
        stats[5 * g.N + n] += uz * uz;
    }
}

}  // namespace lbm
