// Internal interface between the C-ABI runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace lbm {

// Everything a kernel launch needs to know about one context.
struct DevCtx {
    Geo g;
    int codec;            // 0 F64, 1 F32, 2 F16S, 3 BF16S
    void* f;              // in-place population array [19][nz][ny][pitch]
    const uint64_t* mask; // solid bits [nz][ny][wpr]
    void* ghost;          // outflow ghost entries
    const double* prof;   // inflow profiles [6][nz][3] (the per-height base velocities)
    const double* uin;    // per-cell inflow velocities (inflow_slot); what the step kernels read
    const unsigned* odd_list;  // waves of the odd step left to the general kernel
    long long odd_list_n;
    const unsigned* push_list; // canonical indices of the face layer (general-path push)
    long long push_list_n;
    const unsigned* adj_list;  // canonical indices of the two-layer face shell (general-path adjoint)
    long long adj_list_n;
    const int* wave_idx;       // per wave (chunk, row): entry in wave_tab, -1 without solid neighbour
    const uint64_t* wave_tab;  // [entries][18] solid-source masks
    double tau0, c_smag, delta, rho0, force[3];
    double omega[3];      // rotation vector in lattice units (Coriolis); zero: none
    int sponge_w;         // sponge / buffer layer width; 0: off
    double sponge_s;      // its strength s_max
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
    P.target = d.prof;
    return P;
}

// Byte offsets of the population slots a wave touches, fixed per grid and
// codec and computed once per launch on the host (otherwise every wave
// rebuilds them with 64-bit scalar arithmetic).  Slice stride sb = S (padded
// in-place layout) or N (canonical layout) times the store size; d_I is the
// element offset of the neighbour x + c_I.
struct StepOff {
    long long even[NQ];  // I sb: slot I of the own cell
    long long odd[NQ];   // opp(I) sb - d_I: slot opp(I) of the neighbour x - c_I
    long long lo[NQ];    // min(I, opp(I)) sb
    uint32_t on[NQ];     // (opp(I) - lo) sb - d_I, relative to lo (mod 2^32)
    uint32_t oo[NQ];     // (I - lo) sb
};

template <typename T>
static StepOff step_offsets(long long slice, long long rowlen, long long ny)
{
    StepOff o;
    const long long sb = slice * (long long)sizeof(T);
    for (int i = 0; i < NQ; i++) {
        const V3 c = dirv(i);
        const int lo = i < opp(i) ? i : opp(i);
        const long long d = ((long long)c.x + rowlen * (c.y + ny * c.z)) * (long long)sizeof(T);
        o.even[i] = i * sb;
        o.odd[i] = opp(i) * sb - d;
        o.lo[i] = lo * sb;
        o.on[i] = (uint32_t)((opp(i) - lo) * sb - d);
        o.oo[i] = (uint32_t)((i - lo) * sb);
    }
    return o;
}

// Host copy of the odd kernel's test for waves it leaves to the general
// kernel (k_odd in lbm_step.hip applies the same test).
// Rows on a y or z face other than WALL, and chunks holding an x-face cell
// unless the x- face is INFLOW or WALL and the x+ face OUTFLOW or WALL.
__host__ __device__ inline bool odd_wave_is_general(const Geo& g, int cx, int y, int z)
{
    if ((y == 0 && g.face[2] != F_WALL) || (y == g.ny - 1 && g.face[3] != F_WALL)) return true;
    if ((z == 0 && g.face[4] != F_WALL) || (z == g.nz - 1 && g.face[5] != F_WALL)) return true;
    if (cx == 0 && g.face[0] != F_INFLOW && g.face[0] != F_WALL) return true;
    if (cx * 64 + 63 >= g.nx - 1 && g.face[1] != F_OUTFLOW && g.face[1] != F_WALL) return true;
    return false;
}

hipError_t launch_step(const DevCtx& d, int odd, void* stats, hipStream_t s);
hipError_t launch_step_general(const DevCtx& d, int odd, void* stats, hipStream_t s);
hipError_t launch_general_odd(const DevCtx& d, void* stats, hipStream_t s);
hipError_t launch_push(const DevCtx& d, const void* src, void* dst, hipStream_t s);
hipError_t launch_push_cells(const DevCtx& d, const void* src, void* dst, hipStream_t s);
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
hipError_t launch_adjoint(const DevCtx& d, const void* f_t, const void* lam_next, void* lam, const int* probes,
                          int np, const void* probe_src, void* g_inflow, hipStream_t s);

}  // namespace lbm
