// Halo exchange of a slab decomposition along y (the domain splitting of
// the paper's multi-GPU runs): a slab's LBM_HALO side carries a ghost row
// that stands for the neighbour's boundary row.  Only the five populations
// with c_y toward the neighbour cross an interface, once per step:
//   after an even step (swapped layout, slot opp(J) of a cell holds f*_J):
//     pack   the real boundary row's f*_J moving toward the neighbour;
//     unpack into the ghost row's slots opp(J), which the odd step gathers;
//   after an odd step (natural layout, slot J holds f_J(t+1)):
//     pack   the ghost row's slots J that this slab's real cells pushed into;
//     unpack into the real boundary row's slots J, where the pull of J comes
//            from a non-solid ghost cell (else the cell's own bounce-back, or
//            an outflow-copy slot, stays), and into the zero-gradient copies
//            of those slots on OUTFLOW faces.
// One thread per (x, z) of the row; the buffer is [5][nz][nx] in the
// codec's storage type, directions in ascending order.
#include "lbm_device.h"
#include "lbm_launch.h"

#include <type_traits>

namespace lbm {

namespace {

template <int I, int N, class Fn>
__device__ __forceinline__ void halo_for(Fn&& fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        halo_for<I + 1, N>(fn);
    }
}

// Position of direction I among the directions with c_y == CY (ascending).
template <int CY>
constexpr int y_rank(int I)
{
    int k = 0;
    for (int j = 0; j < I; j++)
        if (dirv(j).y == CY) k++;
    return k;
}

// One axis of the pull source of a ghost cell: in range, mirrored at a
// FREESLIP face, wrapped at a PERIODIC one; false across any other face.
__device__ inline bool halo_axis(int& p, int own, int n, int kind_lo, int kind_hi)
{
    if (p >= 0 && p < n) return true;
    const int kind = p < 0 ? kind_lo : kind_hi;
    if (kind == F_FREESLIP) p = own;
    else if (kind == F_PERIODIC) p = p < 0 ? n - 1 : 0;
    else return false;
    return true;
}

// side 0 (y-): ghost row 0, real row 1, sends c_y = -1, receives c_y = +1;
// side 1 (y+): ghost row ny - 1, real row ny - 2, sends +1, receives -1.
template <int K, int SIDE, int UNPACK, int PHASE>
__global__ void __launch_bounds__(256)
k_halo(typename Codec<K>::store* __restrict__ f, const uint64_t* __restrict__ mask, Geo g, Lay L,
       typename Codec<K>::store* __restrict__ buf)
{
    const long long t = blockIdx.x * 256ll + threadIdx.x;
    const int x = (int)(t % g.nx), z = (int)(t / g.nx);
    if (z >= g.nz) return;
    const int ghost = SIDE == 0 ? 0 : g.ny - 1;
    const int real = SIDE == 0 ? 1 : g.ny - 2;
    constexpr int CY = (SIDE == 0) == (UNPACK == 0) ? -1 : 1;   // the directions this call moves
    const bool own_solid = UNPACK && PHASE == 0 && solid_at(mask, g, x, real, z);
    halo_for<1, NQ>([&](auto ic) {
        constexpr int J = decltype(ic)::value;
        constexpr V3 c = dirv(J);
        if constexpr (c.y == CY) {
            constexpr int k = y_rank<CY>(J);
            const long long b = ((long long)k * g.nz + z) * g.nx + x;
            if constexpr (!UNPACK) {
                if constexpr (PHASE == 1) buf[b] = f[pop_index(L, opp(J), x, real, z)];
                else buf[b] = f[pop_index(L, J, x, ghost, z)];
            } else if constexpr (PHASE == 1) {
                f[pop_index(L, opp(J), x, ghost, z)] = buf[b];
            } else {
                if (own_solid) return;
                int px = x - c.x, pz = z - c.z;
                if (!halo_axis(px, x, g.nx, g.face[0], g.face[1])) return;
                if (!halo_axis(pz, z, g.nz, g.face[4], g.face[5])) return;
                if (solid_at(mask, g, px, ghost, pz)) return;
                const typename Codec<K>::store v = buf[b];
                f[pop_index(L, J, x, real, z)] = v;
                // the odd step already applied the zero-gradient outflow copy
                // of this slot (f_J of the face cell one layer out, for J
                // entering through an OUTFLOW x or z face) from the value
                // being replaced: apply it again
                int ox = -1, oz = -1;
                if constexpr (c.x == -1) { if (g.face[1] == F_OUTFLOW && x == g.nx - 2) ox = g.nx - 1; }
                if constexpr (c.x == 1) { if (g.face[0] == F_OUTFLOW && x == 1) ox = 0; }
                if constexpr (c.z == -1) { if (g.face[5] == F_OUTFLOW && z == g.nz - 2) oz = g.nz - 1; }
                if constexpr (c.z == 1) { if (g.face[4] == F_OUTFLOW && z == 1) oz = 0; }
                if (ox >= 0 && !solid_at(mask, g, ox, real, z) && inflow_face_of(g, ox, real, z) < 0)
                    f[pop_index(L, J, ox, real, z)] = v;
                if (oz >= 0 && !solid_at(mask, g, x, real, oz) && inflow_face_of(g, x, real, oz) < 0)
                    f[pop_index(L, J, x, real, oz)] = v;
            }
        }
    });
}

template <int K, int SIDE, int UNPACK>
hipError_t halo_k(const DevCtx& d, int phase, void* buf, hipStream_t s)
{
    using T = typename Codec<K>::store;
    const unsigned blocks = (unsigned)(((long long)d.g.nx * d.g.nz + 255) / 256);
    const Lay L{d.g.S, d.g.pitch, d.g.lrb, d.g.nyp};
    if (phase)
        hipLaunchKernelGGL((k_halo<K, SIDE, UNPACK, 1>), dim3(blocks), dim3(256), 0, s, (T*)d.f, d.mask, d.g, L, (T*)buf);
    else
        hipLaunchKernelGGL((k_halo<K, SIDE, UNPACK, 0>), dim3(blocks), dim3(256), 0, s, (T*)d.f, d.mask, d.g, L, (T*)buf);
    return hipGetLastError();
}

template <int K>
hipError_t halo_codec(const DevCtx& d, int side, int phase, int unpack, void* buf, hipStream_t s)
{
    if (side == 0) return unpack ? halo_k<K, 0, 1>(d, phase, buf, s) : halo_k<K, 0, 0>(d, phase, buf, s);
    return unpack ? halo_k<K, 1, 1>(d, phase, buf, s) : halo_k<K, 1, 0>(d, phase, buf, s);
}

static_assert(y_rank<1>(17) == 4 && y_rank<-1>(18) == 4, "five crossing directions per side");

}  // namespace

hipError_t launch_halo(const DevCtx& d, int side, int phase, int unpack, void* buf, hipStream_t s)
{
    switch (d.codec) {
        case 0: return halo_codec<0>(d, side, phase, unpack, buf, s);
        case 1: return halo_codec<1>(d, side, phase, unpack, buf, s);
        case 2: return halo_codec<2>(d, side, phase, unpack, buf, s);
        case 3: return halo_codec<3>(d, side, phase, unpack, buf, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
