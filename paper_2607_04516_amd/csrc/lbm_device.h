// Device-side building blocks of the D3Q19 LBM-LES library for gfx950:
// the velocity set, storage codecs, the boundary resolution of one
// population, and the local BGK + Smagorinsky collision
// (arXiv 2607.04516, App. D, eqs. D.1-D.11).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int NQ = 19;

struct V3 {
    int x, y, z;
};

// D3Q19 velocities: rest, +-x, +-y, +-z, then +-(1,1,0), +-(1,0,1), +-(0,1,1),
// +-(1,-1,0), +-(1,0,-1), +-(0,1,-1).  Directions 2k-1 and 2k are opposite.
__host__ __device__ constexpr V3 dirv(int i)
{
    const V3 t[NQ] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                      {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, 0, 1},
                      {-1, 0, -1}, {0, 1, 1}, {0, -1, -1}, {1, -1, 0}, {-1, 1, 0},
                      {1, 0, -1}, {-1, 0, 1}, {0, 1, -1}, {0, -1, 1}};
    return t[i];
}

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

__host__ __device__ constexpr int comp(V3 v, int a) { return a == 0 ? v.x : (a == 1 ? v.y : v.z); }

__host__ __device__ constexpr int dir_index(int x, int y, int z)
{
    for (int i = 0; i < NQ; i++) {
        V3 v = dirv(i);
        if (v.x == x && v.y == y && v.z == z) return i;
    }
    return -1;
}

// Direction with the components selected by the bit mask m (bit a = axis a) negated.
__host__ __device__ constexpr int mirrored(int i, int m)
{
    V3 v = dirv(i);
    return dir_index((m & 1) ? -v.x : v.x, (m & 2) ? -v.y : v.y, (m & 4) ? -v.z : v.z);
}

// Position k (0..4) of direction i among the five directions whose component
// a equals s, in increasing direction order (-1 when comp(i, a) != s).
__host__ __device__ constexpr int entering_rank(int i, int a, int s)
{
    int k = 0;
    for (int j = 0; j < NQ; j++) {
        if (comp(dirv(j), a) != s) continue;
        if (j == i) return k;
        k++;
    }
    return -1;
}

template <typename T>
__host__ __device__ constexpr T weight(int i)
{
    return i == 0 ? T(1) / T(3) : (i <= 6 ? T(1) / T(18) : T(1) / T(36));
}

// Face kinds (same values as enum lbm_face_kind in lbm.h).
enum { F_PERIODIC = 0, F_INFLOW = 1, F_OUTFLOW = 2, F_FREESLIP = 3, F_WALL = 4 };

// --------------------------------------------------------------------------
// Storage codecs: what one population occupies in HBM.  The stored quantity
// is always the shift h = f - w*rho0 (times a power-of-two scale for binary16
// so that the values sit in its normal range).
// --------------------------------------------------------------------------
template <int K>
struct Codec;

// dec/enc convert to and from the true shift h; raw/pack convert without
// the scale (the step kernels work in stored units, SC times h).
template <>
struct Codec<0> {  // FP64
    using store = double;
    using real = double;
    static constexpr int SC = 1;
    __device__ static real dec(store v) { return v; }
    __device__ static store enc(real v) { return v; }
    __device__ static real raw(store v) { return v; }
    __device__ static store pack(real v) { return v; }
};

template <>
struct Codec<1> {  // FP32
    using store = float;
    using real = float;
    static constexpr int SC = 1;
    __device__ static real dec(store v) { return v; }
    __device__ static store enc(real v) { return v; }
    __device__ static real raw(store v) { return v; }
    __device__ static store pack(real v) { return v; }
};

template <>
struct Codec<2> {  // IEEE binary16, round to nearest even, scaled by 2^8
    using store = _Float16;
    using real = float;
    static constexpr int SC = 256;
    __device__ static real dec(store v) { return float(v) * (1.0f / SC); }
    __device__ static store enc(real v) { return store(v * float(SC)); }
    __device__ static real raw(store v) { return float(v); }
    __device__ static store pack(real v) { return store(v); }
};

template <>
struct Codec<3> {  // bfloat16, round to nearest even
    using store = uint16_t;
    using real = float;
    static constexpr int SC = 1;
    __device__ static real dec(store v) { return __uint_as_float(uint32_t(v) << 16); }
    __device__ static store enc(real v)
    {
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return store(u >> 16);
    }
    __device__ static real raw(store v) { return dec(v); }
    __device__ static store pack(real v) { return enc(v); }
};

// --------------------------------------------------------------------------
// Geometry and parameters (passed by value to every kernel).
// --------------------------------------------------------------------------
struct Geo {
    int nx, ny, nz;
    int pitch;           // x pitch of the in-place population array (multiple of 64)
    int lrb;             // log2 of the rows per block of the in-place array (row blocks, below)
    int nyp;             // rows per z plane of the in-place array: ny rounded up to whole blocks
    int wpr;             // 64-bit mask words per row
    int ncx;             // 64-cell chunks per row = pitch / 64
    int face[6];         // face kinds, order x-, x+, y-, y+, z-, z+
    long long S;         // pitch*nyp*nz: elements of one population over the grid
    long long N;         // nx*ny*nz
    long long ghost_off[6];  // element offset of each outflow face's ghost block
    long long in_off[6];     // first per-cell inflow entry of each INFLOW_EQ face (-1: none)
};

// Entry i of a six-entry Geo array for a runtime i, as a select chain.  Where
// a kernel indexes a kernel-argument array with a runtime index the compiler
// may copy the whole Geo into scratch memory in every thread; which form
// avoids that depends on the call site (the build test checks the hot
// kernels for scratch).
template <typename T>
__host__ __device__ inline T pick6(const T (&v)[6], int i)
{
    return i == 0 ? v[0] : i == 1 ? v[1] : i == 2 ? v[2] : i == 3 ? v[3] : i == 4 ? v[4] : v[5];
}

// Per-cell inflow velocities (the boundary velocity array): three doubles
// per cell of every INFLOW_EQ face, faces stacked from x- to z+; an x face is
// indexed y + ny z, a y face x + nx z, a z face x + nx y.
__host__ __device__ inline long long inflow_slot(const Geo& g, int F, int x, int y, int z)
{
    const int a = F >> 1;
    const long long j = a == 0 ? y + (long long)g.ny * z : a == 1 ? x + (long long)g.nx * z : x + (long long)g.nx * y;
    return pick6(g.in_off, F) + j;
}

template <typename R>
__device__ inline void load_inflow(const double* __restrict__ uin, const Geo& g, int F, int x, int y, int z, R& ux,
                                   R& uy, R& uz)
{
    const double* p = uin + 3 * inflow_slot(g, F, x, y, z);
    ux = R(p[0]);
    uy = R(p[1]);
    uz = R(p[2]);
}

template <typename R>
struct Phys {
    R tau0;
    R ksmag;       // 18 (C Delta)^2 = 2 (C Delta)^2 / cs^4
    R rho0;
    R F[3];        // uniform body force
    R W2[3];       // 2 Omega, Omega the rotation vector in lattice units (Coriolis)
    int has_rot;   // W2 != 0
    int has_force; // F != 0 or has_rot: the Guo source is applied
    int sponge_w;  // width W of the sponge / buffer layers; 0: off
    R sponge_s;    // strength s_max at the layer next to the face
    const double* target;  // per-cell boundary states of the INFLOW_EQ faces (inflow_slot): the nudging targets
};

// Body force on one cell: the uniform force plus the Coriolis force of the
// rotating frame (App. E), F_c = -2 rho Omega x u0 = -2 Omega x m, with
// m = sum c f the momentum recovered before the force enters (the stored
// shift w rho0 carries no momentum, so the shifted sums give m directly).
// Contraction is off so every kernel that inlines this rounds alike.
template <typename R>
__device__ inline void cell_force(const Phys<R>& P, R mx, R my, R mz, R& Fx, R& Fy, R& Fz)
{
#pragma clang fp contract(off)
    Fx = P.F[0];
    Fy = P.F[1];
    Fz = P.F[2];
    if (P.has_rot) {
        Fx = Fx - (P.W2[1] * mz - P.W2[2] * my);
        Fy = Fy - (P.W2[2] * mx - P.W2[0] * mz);
        Fz = Fz - (P.W2[0] * my - P.W2[1] * mx);
    }
}

// Layout of one population array.  Rows are numbered row = y + nyr*z, nyr
// the rows per z plane in memory.
//   plain (lrb < 0): slices, nyr = ny, index = dir*S + x + pitch*row;
//   row blocks (lrb >= 0): R = 2^lrb consecutive rows hold their 19
//     populations together, [row / R][dir][row % R][pitch]: index =
//     ((row / R * 19 + dir) * R + row % R) * pitch + x.  nyr is ny rounded
//     up to a multiple of R (the rows beyond ny are padding no kernel
//     touches), so a neighbour in z sits nyr / R blocks away at the same
//     place in its block.
// The in-place array of a context uses row blocks (the 19 streams of a
// step then fall into a few MiB instead of 19 slices 0.3 GiB apart, which
// the DRAM serves measurably faster); canonical arrays are plain slices.
struct Lay {
    long long S;  // plain: slice stride in elements
    int pitch;    // row length in elements
    int lrb;      // log2 rows per block; -1: plain slices
    int nyr;      // rows per z plane
};

__host__ __device__ inline long long pop_index_row(const Lay& L, int dir, long long row, int x)
{
    if (L.lrb < 0) return (long long)dir * L.S + row * L.pitch + x;
    const long long rmask = (1ll << L.lrb) - 1;
    return ((((row >> L.lrb) * NQ + dir) << L.lrb) + (row & rmask)) * L.pitch + x;
}

__host__ __device__ inline long long pop_index(const Lay& L, int dir, int x, int y, int z)
{
    return pop_index_row(L, dir, (long long)y + (long long)L.nyr * z, x);
}

__device__ inline bool solid_at(const uint64_t* __restrict__ mask, const Geo& g, int x, int y, int z)
{
    uint64_t w = mask[(long long)(y + (long long)g.ny * z) * g.wpr + (x >> 6)];
    return (w >> (x & 63)) & 1ull;
}

__device__ inline int dimn(const Geo& g, int a) { return a == 0 ? g.nx : (a == 1 ? g.ny : g.nz); }

// Lowest-numbered inflow face whose layer holds (x,y,z), or -1.
__host__ __device__ inline int inflow_face_of(const Geo& g, int x, int y, int z)
{
    if (g.face[0] == F_INFLOW && x == 0) return 0;
    if (g.face[1] == F_INFLOW && x == g.nx - 1) return 1;
    if (g.face[2] == F_INFLOW && y == 0) return 2;
    if (g.face[3] == F_INFLOW && y == g.ny - 1) return 3;
    if (g.face[4] == F_INFLOW && z == 0) return 4;
    if (g.face[5] == F_INFLOW && z == g.nz - 1) return 5;
    return -1;
}

// --------------------------------------------------------------------------
// Boundary resolution of direction I at a non-solid cell p = (x,y,z).
//
// The streaming (eq. D.3) pulls f_I(p, t+1) = f*_j(s, t) with s = p - c_I,
// j = I, and the face rules for each axis the pull leaves the grid through:
//   WALL      halfway bounce-back: the value is f*_opp(I)(p)
//   PERIODIC  s wraps
//   FREESLIP  specular reflection: j mirrors that component, s_a = p_a
//   INFLOW / OUTFLOW never crossed by a pull from a fluid cell
// and halfway bounce-back when s is solid (App. D, last paragraph).
//
// The same slot serves the pull of direction I and the push of direction
// opp(I) (the streaming rules are time reversible), which is what makes the
// in-place A-A update race free.  Res.kind:
//   0  slot (x,y,z,dir): the pull reads the post-collision value stored at
//      (s, opp(j)) in the swapped layout; bounce-back gives (p, I)
//   2  no slot: the pull leaves through an inflow or outflow face
// --------------------------------------------------------------------------
struct Res {
    int kind;
    int x, y, z;
    int dir;
    int vx, vy, vz;  // velocity of direction dir
};

template <int I>
__device__ inline Res resolve_plain(const Geo& g, const uint64_t* __restrict__ mask, int x, int y, int z)
{
    constexpr V3 c = dirv(I);
    int s[3] = {x - c.x, y - c.y, z - c.z};
    const int p[3] = {x, y, z};
    int m = 0;  // mirrored axes
    Res r;
    r.kind = 0;
    r.x = x; r.y = y; r.z = z; r.dir = I;  // valid in-bounds slot even when kind == 2
    r.vx = c.x; r.vy = c.y; r.vz = c.z;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int ca = comp(c, a);
        if (ca == 0) continue;
        const int n = dimn(g, a);
        const bool lo = (s[a] < 0), hi = (s[a] >= n);
        if (!(lo || hi)) continue;
        const int kind = lo ? g.face[2 * a] : g.face[2 * a + 1];
        if (kind == F_WALL) {
            return r;
        } else if (kind == F_PERIODIC) {
            s[a] = lo ? s[a] + n : s[a] - n;
        } else if (kind == F_FREESLIP) {
            m |= (1 << a);
            s[a] = p[a];
        } else {
            r.kind = 2;
            return r;
        }
    }
    if (solid_at(mask, g, s[0], s[1], s[2])) return r;
    // j = I with the mirrored components flipped; the value sits in slot opp(j)
    constexpr int o0 = opp(mirrored(I, 0)), o1 = opp(mirrored(I, 1)), o2 = opp(mirrored(I, 2)),
                  o3 = opp(mirrored(I, 3)), o4 = opp(mirrored(I, 4)), o5 = opp(mirrored(I, 5)),
                  o6 = opp(mirrored(I, 6)), o7 = opp(mirrored(I, 7));
    int d;
    switch (m) {
        case 0: d = o0; break;
        case 1: d = o1; break;
        case 2: d = o2; break;
        case 3: d = o3; break;
        case 4: d = o4; break;
        case 5: d = o5; break;
        case 6: d = o6; break;
        default: d = o7; break;
    }
    r.x = s[0]; r.y = s[1]; r.z = s[2]; r.dir = d;
    // slot opp(j): velocity -c_j, j = I with the mirrored components negated
    r.vx = (m & 1) ? c.x : -c.x;
    r.vy = (m & 2) ? c.y : -c.y;
    r.vz = (m & 4) ? c.z : -c.z;
    return r;
}

// Zero-gradient outflow: when direction I enters through an outflow face at
// p, f_I(p) copies what the cell q (p moved one layer inward along every such
// face) receives.  Returns true in that case with q and the lowest-numbered
// such face (the owner of the ghost entry).
template <int I>
__device__ inline bool outflow_entering(const Geo& g, int x, int y, int z, int& qx, int& qy, int& qz, int& owner)
{
    constexpr V3 c = dirv(I);
    bool moved = false;
    owner = 6;
    qx = x; qy = y; qz = z;
    if (c.x == 1 && g.face[0] == F_OUTFLOW && x == 0) { qx = 1; moved = true; owner = min(owner, 0); }
    if (c.x == -1 && g.face[1] == F_OUTFLOW && x == g.nx - 1) { qx = g.nx - 2; moved = true; owner = min(owner, 1); }
    if (c.y == 1 && g.face[2] == F_OUTFLOW && y == 0) { qy = 1; moved = true; owner = min(owner, 2); }
    if (c.y == -1 && g.face[3] == F_OUTFLOW && y == g.ny - 1) { qy = g.ny - 2; moved = true; owner = min(owner, 3); }
    if (c.z == 1 && g.face[4] == F_OUTFLOW && z == 0) { qz = 1; moved = true; owner = min(owner, 4); }
    if (c.z == -1 && g.face[5] == F_OUTFLOW && z == g.nz - 1) { qz = g.nz - 2; moved = true; owner = min(owner, 5); }
    return moved;
}

// Index of the ghost entry for (face, direction I, cell p).  With AT the
// face's first entry is goff instead of g.ghost_off[face] (a caller whose
// face index is not a kernel argument passes it in, so that the by-value
// descriptor is not indexed at run time).
template <int I, bool AT = false>
__device__ inline long long ghost_index(const Geo& g, int face, int x, int y, int z, long long goff = 0)
{
    const int a = face >> 1;
    const int s = (face & 1) ? -1 : 1;
    int k;
    long long cell;
    if (a == 0) { k = entering_rank(I, 0, s); cell = y + (long long)g.ny * z; }
    else if (a == 1) { k = entering_rank(I, 1, s); cell = x + (long long)g.nx * z; }
    else { k = entering_rank(I, 2, s); cell = x + (long long)g.nx * y; }
    long long fc = (a == 0) ? (long long)g.ny * g.nz : (a == 1 ? (long long)g.nx * g.nz : (long long)g.nx * g.ny);
    if constexpr (AT) return goff + (long long)k * fc + cell;
    else return g.ghost_off[face] + (long long)k * fc + cell;
}

// Full resolution of the pull of direction I at a fluid (non-solid,
// non-inflow) cell, outflow copy included; kind 0 slot in the swapped layout.
template <int I>
__device__ inline Res resolve_full(const Geo& g, const uint64_t* __restrict__ mask, int x, int y, int z)
{
    int qx, qy, qz, owner;
    if (outflow_entering<I>(g, x, y, z, qx, qy, qz, owner)) {
        if (solid_at(mask, g, qx, qy, qz)) {
            constexpr V3 c = dirv(I);
            Res r;
            r.kind = 0; r.x = x; r.y = y; r.z = z; r.dir = I;
            r.vx = c.x; r.vy = c.y; r.vz = c.z;
            return r;
        }
        return resolve_plain<I>(g, mask, qx, qy, qz);
    }
    return resolve_plain<I>(g, mask, x, y, z);
}

// --------------------------------------------------------------------------
// Equilibrium of the shifted populations (eq. D.4 minus w_i rho0):
//   heq_i = w_i (rho - rho0) + w_i rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)
// --------------------------------------------------------------------------
template <typename R>
__device__ inline void equilibrium_shifted(R rho, R drho, R ux, R uy, R uz, R* heq)
{
#pragma clang fp contract(off)
    const R usq15 = R(1.5) * fma(ux, ux, fma(uy, uy, uz * uz));
    heq[0] = weight<R>(0) * fma(-rho, usq15, drho);
#pragma unroll
    for (int k = 1; k < NQ; k += 2) {
        const V3 c = dirv(k);
        const R e = R(c.x) * ux + R(c.y) * uy + R(c.z) * uz;
        const R w = weight<R>(k);
        const R even = w * fma(rho, fma(R(4.5) * e, e, -usq15), drho);
        const R odd = w * rho * (R(3) * e);
        heq[k] = even + odd;
        heq[k + 1] = even - odd;
    }
}

// Fast reciprocal and square root: hardware v_rcp_f32 / v_sqrt_f32 (about
// 1 ulp) for float; correctly rounded for double.
template <typename R>
__device__ inline R fast_rcp(R x) { return R(1) / x; }
template <>
__device__ inline float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename R>
__device__ inline R fast_sqrt(R x) { return sqrt(x); }
template <>
__device__ inline float fast_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// --------------------------------------------------------------------------
// The collision of one cell in the form the step kernels use.  h holds the
// stored shifts (SC times f_i - w_i rho0); the update is the same BGK +
// Smagorinsky step as collide() with fewer operations:
//   * opposite pairs enter through s_k = h_i + h_j and d_k = h_i - h_j;
//   * Pi comes from the raw second moment of h and the exact D3Q19
//     identity sum_i c_ia c_ib feq_i = rho (delta_ab/3 + u_a u_b)
//     (4th-order isotropy, App. D), so no per-direction feq is formed;
//   * h*_i = (1 - w) h_i + w heq_i is evaluated per pair from the even and
//     odd parts of heq.
// Returns rho - rho0, u and tau_eff.
// --------------------------------------------------------------------------
// rho - rho0 and u of stored shifts h (SC times the true shifts), in the
// summation order of collide_pairs, so diagnostics match the collision bit
// for bit.  Contraction is off and every fused multiply-add is explicit, so
// the arithmetic is the same in every kernel that inlines it.
template <typename R, int SC>
__device__ inline void moments_pairs(const R* h, const Phys<R>& P, R& drho, R& ux, R& uy, R& uz, R& Fx, R& Fy,
                                     R& Fz)
{
#pragma clang fp contract(off)
    constexpr R isc = R(1) / R(SC);
    const R s1 = h[1] + h[2], d1 = h[1] - h[2];
    const R s2 = h[3] + h[4], d2 = h[3] - h[4];
    const R s3 = h[5] + h[6], d3 = h[5] - h[6];
    const R s4 = h[7] + h[8], d4 = h[7] - h[8];
    const R s5 = h[9] + h[10], d5 = h[9] - h[10];
    const R s6 = h[11] + h[12], d6 = h[11] - h[12];
    const R s7 = h[13] + h[14], d7 = h[13] - h[14];
    const R s8 = h[15] + h[16], d8 = h[15] - h[16];
    const R s9 = h[17] + h[18], d9 = h[17] - h[18];
    const R drs = ((h[0] + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)) + (s8 + s9);
    const R jx = ((d1 + d4) + (d5 + d7)) + d8;
    const R jy = ((d2 + d4) + (d6 - d7)) + d9;
    const R jz = ((d3 + d5) + (d6 - d8)) - d9;
    drho = drs * isc;
    const R irho = fast_rcp<R>(P.rho0 + drho);
    cell_force(P, jx * isc, jy * isc, jz * isc, Fx, Fy, Fz);
    ux = fma(jx, isc, R(0.5) * Fx) * irho;
    uy = fma(jy, isc, R(0.5) * Fy) * irho;
    uz = fma(jz, isc, R(0.5) * Fz) * irho;
}

template <typename R, int SC>
__device__ inline void moments_pairs(const R* h, const Phys<R>& P, R& drho, R& ux, R& uy, R& uz)
{
    R Fx, Fy, Fz;
    moments_pairs<R, SC>(h, P, drho, ux, uy, uz, Fx, Fy, Fz);
}

template <typename R, int SC>
__device__ inline void collide_pairs(R* h, const Phys<R>& P, R& drho_o, R& ux, R& uy, R& uz, R& tau_o)
{
#pragma clang fp contract(off)
    constexpr R isc = R(1) / R(SC);
    const R s1 = h[1] + h[2], d1 = h[1] - h[2];
    const R s2 = h[3] + h[4], d2 = h[3] - h[4];
    const R s3 = h[5] + h[6], d3 = h[5] - h[6];
    const R s4 = h[7] + h[8], d4 = h[7] - h[8];
    const R s5 = h[9] + h[10], d5 = h[9] - h[10];
    const R s6 = h[11] + h[12], d6 = h[11] - h[12];
    const R s7 = h[13] + h[14], d7 = h[13] - h[14];
    const R s8 = h[15] + h[16], d8 = h[15] - h[16];
    const R s9 = h[17] + h[18], d9 = h[17] - h[18];
    const R drs = ((h[0] + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)) + (s8 + s9);
    const R jx = ((d1 + d4) + (d5 + d7)) + d8;
    const R jy = ((d2 + d4) + (d6 - d7)) + d9;
    const R jz = ((d3 + d5) + (d6 - d8)) - d9;
    const R mxx = ((s1 + s4) + (s5 + s7)) + s8;
    const R myy = ((s2 + s4) + (s6 + s7)) + s9;
    const R mzz = ((s3 + s5) + (s6 + s8)) + s9;
    const R mxy = s4 - s7, mxz = s5 - s8, myz = s6 - s9;
    const R drho = drs * isc;
    const R rho = P.rho0 + drho;
    const R irho = fast_rcp<R>(rho);
    R Fx, Fy, Fz;
    cell_force(P, jx * isc, jy * isc, jz * isc, Fx, Fy, Fz);
    ux = fma(jx, isc, R(0.5) * Fx) * irho;
    uy = fma(jy, isc, R(0.5) * Fy) * irho;
    uz = fma(jz, isc, R(0.5) * Fz) * irho;
    // Pi = M - (drho/3) I - rho u u  (exact D3Q19 identity for sum c c feq)
    const R t3 = drho * R(1.0 / 3.0);
    const R rux = rho * ux, ruy = rho * uy;
    const R pxx = fma(-rux, ux, fma(mxx, isc, -t3));
    const R pyy = fma(-ruy, uy, fma(myy, isc, -t3));
    const R pzz = fma(-rho * uz, uz, fma(mzz, isc, -t3));
    const R pxy = fma(-rux, uy, mxy * isc);
    const R pxz = fma(-rux, uz, mxz * isc);
    const R pyz = fma(-ruy, uz, myz * isc);
    const R pd = fma(pxx, pxx, fma(pyy, pyy, pzz * pzz));
    const R po = fma(pxy, pxy, fma(pxz, pxz, pyz * pyz));
    const R q = fast_sqrt<R>(R(2) * fma(R(2), po, pd));
    const R tau = R(0.5) * (P.tau0 + fast_sqrt<R>(fma(P.ksmag * q, irho, P.tau0 * P.tau0)));
    const R om = fast_rcp<R>(tau);
    const R om1 = R(1) - om;
    // heq_i = w_i [drho - 1.5 rho u.u] + w_i rho (4.5 e^2 +- 3 e), times SC
    const R usq = fma(ux, ux, fma(uy, uy, uz * uz));
    const R base = fma(R(-1.5) * rho, usq, drho);
    const R a0 = om * R(SC) * weight<R>(0), af = om * R(SC) * weight<R>(1), ae = om * R(SC) * weight<R>(7);
    const R c0 = a0 * base, cf = af * base, ce = ae * base;
    const R bf = af * R(4.5) * rho, be = ae * R(4.5) * rho;
    const R gf = af * R(3) * rho, ge = ae * R(3) * rho;
    h[0] = fma(om1, h[0], c0);
#define LBM_PAIR(i, e, C, B, G)                 \
    {                                           \
        const R ee = (e);                       \
        const R t = fma((B), ee * ee, (C));     \
        const R o = (G) * ee;                   \
        h[i] = fma(om1, h[i], t + o);           \
        h[i + 1] = fma(om1, h[i + 1], t - o);   \
    }
    LBM_PAIR(1, ux, cf, bf, gf)
    LBM_PAIR(3, uy, cf, bf, gf)
    LBM_PAIR(5, uz, cf, bf, gf)
    LBM_PAIR(7, ux + uy, ce, be, ge)
    LBM_PAIR(9, ux + uz, ce, be, ge)
    LBM_PAIR(11, uy + uz, ce, be, ge)
    LBM_PAIR(13, ux - uy, ce, be, ge)
    LBM_PAIR(15, ux - uz, ce, be, ge)
    LBM_PAIR(17, uy - uz, ce, be, ge)
#undef LBM_PAIR
    if (P.has_force) {
        // Guo source (1 - w/2) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F, times SC
        const R pre = (R(1) - R(0.5) * om) * R(SC);
        const R uF = fma(ux, Fx, fma(uy, Fy, uz * Fz));
        h[0] = fma(pre * weight<R>(0), R(-3) * uF, h[0]);
#pragma unroll
        for (int i = 1; i < NQ; i += 2) {
            const V3 c = dirv(i);
            const R e = R(c.x) * ux + R(c.y) * uy + R(c.z) * uz;
            const R cF = R(c.x) * Fx + R(c.y) * Fy + R(c.z) * Fz;
            const R ev = pre * weight<R>(i) * (R(9) * e * cF - R(3) * uF);
            const R od = pre * weight<R>(i) * (R(3) * cF);
            h[i] += ev + od;
            h[i + 1] += ev - od;
        }
    }
    drho_o = drho;
    tau_o = tau;
}

// Sponge and buffer nudging after the collision: next to every INFLOW_EQ
// face except the ground, a cell at distance d = 1..W from the face layer
// has strength s = s_max ((W + 1 - d) / W)^2 (the largest over the faces,
// the lower-numbered face on ties), and its populations move by
// s (feq(rho, u_t) - feq(rho, u)), u_t the face's profile at the cell's
// height (the top row for z+).  The density parts of the two equilibria
// cancel, so the shift is w rho [-1.5 (|u_t|^2 - |u|^2) + 4.5 (e_t^2 - e^2)
// + 3 (e_t - e)] per direction, times s and the storage scale.
template <typename R, int SC>
__device__ inline void nudge_at(R* h, const Phys<R>& P, const Geo& g, int x, int y, int z, R drho, R ux, R uy,
                                R uz)
{
    const int dist[6] = {x, g.nx - 1 - x, y, g.ny - 1 - y, z, g.nz - 1 - z};
    R best = R(0);
    int face = -1;
#pragma unroll
    for (int F = 0; F < 6; F++) {
        if (F == 4 || g.face[F] != F_INFLOW) continue;
        const int d = dist[F];
        if (d < 1 || d > P.sponge_w) continue;
        const R r = R(P.sponge_w + 1 - d) / R(P.sponge_w);
        const R s = P.sponge_s * r * r;
        if (s > best) {
            best = s;
            face = F;
        }
    }
    if (face < 0) return;
    // the face's boundary state at the cell's projection onto the face
    const double* pt = P.target + 3 * inflow_slot(g, face, x, y, z);
    const R tx = R(pt[0]), ty = R(pt[1]), tz = R(pt[2]);
    const R k = best * R(SC) * (P.rho0 + drho);
    const R dus = R(-1.5) * ((tx * tx + ty * ty + tz * tz) - (ux * ux + uy * uy + uz * uz));
    h[0] += k * weight<R>(0) * dus;
#pragma unroll
    for (int i = 1; i < NQ; i += 2) {
        const V3 c = dirv(i);
        const R et = R(c.x) * tx + R(c.y) * ty + R(c.z) * tz;
        const R e = R(c.x) * ux + R(c.y) * uy + R(c.z) * uz;
        const R ev = weight<R>(i) * (dus + R(4.5) * (et * et - e * e));
        const R od = weight<R>(i) * (R(3) * (et - e));
        h[i] += k * (ev + od);
        h[i + 1] += k * (ev - od);
    }
}

// The collision of one interior cell at (x, y, z), nudging included.
template <typename R, int SC>
__device__ inline void collide_at(R* h, const Phys<R>& P, const Geo& g, int x, int y, int z, R& drho, R& ux, R& uy,
                                  R& uz, R& tau)
{
    collide_pairs<R, SC>(h, P, drho, ux, uy, uz, tau);
    if (P.sponge_w > 0) nudge_at<R, SC>(h, P, g, x, y, z, drho, ux, uy, uz);
}

// --------------------------------------------------------------------------
// Wave-level helpers for kernels where one wave is one 64-cell chunk of a
// row (x = 64 cx + lane): the bit-packed solid mask then gives, per row, one
// 64-bit word whose bit l is lane l's cell.
// --------------------------------------------------------------------------
// The solid mask is read-only while a kernel runs: reading it through the
// constant address space lets wave-uniform words come in by scalar loads.
typedef const uint64_t __attribute__((address_space(4))) const_u64;

__device__ inline uint64_t mask_word(const uint64_t* mask, long long i)
{
    return ((const const_u64*)mask)[i];
}

typedef const int __attribute__((address_space(4))) const_i32;

// Solid-source masks of one wave (64 cells of a row) for directions 1..18,
// bit l set when the pull source of lane l is solid (WALL faces included),
// read from a per-grid table built once (see build_wave_masks): a wave with
// no solid neighbour has no entry.  Wave-uniform, so scalar loads.
struct WaveMask {
    const uint64_t* m;  // 18 words, or nullptr
    template <int I>
    __device__ uint64_t get() const
    {
        return m ? ((const const_u64*)m)[I - 1] : 0ull;
    }
};

__device__ inline WaveMask wave_mask(const int* __restrict__ idx, const uint64_t* __restrict__ tab, long long wave)
{
    const int k = ((const const_i32*)idx)[wave];
    WaveMask w;
    w.m = k >= 0 ? tab + 18ll * k : nullptr;
    return w;
}

// A wave-uniform 64-bit value, made explicitly uniform (readfirstlane of
// each half; the builtin returns int, so go through uint32_t before
// widening or the low half would be sign-extended).
__device__ inline uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Per-lane select of a 32-bit value by a wave-uniform 64-bit lane mask (bit
// l picks b for lane l): one v_cndmask with the mask in an SGPR pair.
__device__ inline uint32_t lane_select(uint32_t a, uint32_t b, uint64_t m)
{
    // m is wave-uniform by construction; readfirstlane makes that explicit
    // so that it is held in an SGPR pair
    const uint64_t ms = uniform_u64(m);
    uint32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(ms));
    return r;
}


// Solid words of the 3 x 3 rows around (y, z) (each interior), chunks
// cx - 1, cx, cx + 1 (0 beyond the row).  Index [dz + 1][dy + 1].
struct RowWin {
    uint64_t p[3][3], c[3][3], n[3][3];
};

// A WALL face acts as a layer of solid cells just outside the grid (halfway
// bounce-back at the face plane is the same rule as at a solid neighbour),
// so rows and columns beyond WALL faces read as all-solid words.  Callers
// only ask for rows beyond WALL faces.
__device__ inline void load_rows(RowWin& W, const uint64_t* mask, const Geo& g, int cx, int y, int z)
{
    const bool xm_wall = g.face[0] == F_WALL, xp_wall = g.face[1] == F_WALL;
    const bool last = (cx + 1 >= g.wpr);
    const int l_last = (g.nx - 1) - cx * 64;  // lane of x = nx - 1 when this chunk holds it
    const uint64_t pad = (xp_wall && last && l_last < 63) ? (~0ull << (l_last + 1)) : 0ull;
    // Every word is computed as a value (loads from a clamped, always valid
    // index, then selects), never stored under a branch: that keeps the
    // window in scalar registers instead of a private (scratch) array.
    // A row beyond a FREESLIP face is the face row itself (the mirrored pull
    // source lies in the cell's own row); beyond a WALL face it is all solid.
#pragma unroll
    for (int dz = -1; dz <= 1; dz++)
#pragma unroll
        for (int dy = -1; dy <= 1; dy++) {
            int yy = y + dy, zz = z + dz;
            if (yy < 0 && g.face[2] == F_FREESLIP) yy = 0;
            if (yy >= g.ny && g.face[3] == F_FREESLIP) yy = g.ny - 1;
            if (zz < 0 && g.face[4] == F_FREESLIP) zz = 0;
            if (zz >= g.nz && g.face[5] == F_FREESLIP) zz = g.nz - 1;
            const bool out = yy < 0 || yy >= g.ny || zz < 0 || zz >= g.nz;
            const long long w = out ? (long long)cx : ((long long)yy + (long long)g.ny * zz) * g.wpr + cx;
            const uint64_t wc = mask_word(mask, w);
            const uint64_t wp = mask_word(mask, cx > 0 ? w - 1 : w);
            const uint64_t wn = mask_word(mask, !last ? w + 1 : w);
            W.c[dz + 1][dy + 1] = out ? ~0ull : (wc | pad);
            W.p[dz + 1][dy + 1] = out ? ~0ull : (cx > 0 ? wp : (xm_wall ? ~0ull : 0ull));
            W.n[dz + 1][dy + 1] = out ? ~0ull : (!last ? wn : (xp_wall ? ~0ull : 0ull));
        }
}

// The box of cells the fast kernels take (inclusive bounds): every cell at
// least L layers inside each face, L = 0 for WALL faces (bounce-back, like
// solid cells) and FREESLIP faces (a per-row remap of the crossing
// directions, see row_class), 1 for PERIODIC faces, and 1 (push) or 2
// (adjoint: outflow copies and inflow cells reach one layer further) for
// INFLOW and OUTFLOW faces.  The rest runs the general code.
struct Box {
    int x0, x1, y0, y1, z0, z1;
};

__host__ __device__ inline int face_layers(int kind, int adjoint)
{
    if (kind == F_WALL || kind == F_FREESLIP) return 0;
    if (kind == F_INFLOW || kind == F_OUTFLOW) return adjoint ? 2 : 1;
    return 1;
}

// Whether the adjoint's wave blocks take the x-face layers of their rows
// too (an INFLOW x- face and an OUTFLOW x+ face; per-lane rules in the
// adjoint kernel).
__host__ __device__ inline bool adj_x_edges(const Geo& g)
{
    return g.face[0] == F_INFLOW && g.face[1] == F_OUTFLOW && g.nx >= 4;
}

// Whether the push kernel's wave blocks take the x-face cells of row (y, z)
// too: an INFLOW x- face and an OUTFLOW x+ face, 32-bit or wider storage,
// and a row not next to an INFLOW y or z face.
__host__ __device__ inline bool push_x_edge_row(const Geo& g, int wide, int y, int z)
{
    return wide && g.face[0] == F_INFLOW && g.face[1] == F_OUTFLOW && g.nx >= 4 &&
           !(g.face[2] == F_INFLOW && y == 1) && !(g.face[3] == F_INFLOW && y == g.ny - 2) &&
           !(g.face[4] == F_INFLOW && z == 1) && !(g.face[5] == F_INFLOW && z == g.nz - 2);
}

// Row class of the fast kernels: 3 cy + cz with cy = 1 (2) for the y = 0
// (y = ny - 1) row of a FREESLIP face, else 0, and cz likewise for z.  In
// such a row every direction that crosses the face pulls the mirrored
// direction from the neighbour in the cell's own row (specular reflection at
// the face plane), a wave-uniform change of slot and offset.
__host__ __device__ inline int row_class(const Geo& g, int y, int z)
{
    const int cy = (y == 0 && g.face[2] == F_FREESLIP) ? 1 : ((y == g.ny - 1 && g.face[3] == F_FREESLIP) ? 2 : 0);
    const int cz = (z == 0 && g.face[4] == F_FREESLIP) ? 1 : ((z == g.nz - 1 && g.face[5] == F_FREESLIP) ? 2 : 0);
    return 3 * cy + cz;
}

__host__ __device__ inline Box main_box(const Geo& g, int adjoint)
{
    Box b;
    b.x0 = face_layers(g.face[0], adjoint);
    b.x1 = g.nx - 1 - face_layers(g.face[1], adjoint);
    b.y0 = face_layers(g.face[2], adjoint);
    b.y1 = g.ny - 1 - face_layers(g.face[3], adjoint);
    b.z0 = face_layers(g.face[4], adjoint);
    b.z1 = g.nz - 1 - face_layers(g.face[5], adjoint);
    return b;
}

// Bit l set when the pull source (64 cx + l) - c_I of direction I is solid.
template <int I>
__device__ inline uint64_t solid_src_mask(const RowWin& W)
{
    constexpr V3 c = dirv(I);
    const uint64_t wc = W.c[1 - c.z][1 - c.y];
    if constexpr (c.x == 1) return (wc << 1) | (W.p[1 - c.z][1 - c.y] >> 63);
    else if constexpr (c.x == -1) return (wc >> 1) | (W.n[1 - c.z][1 - c.y] << 63);
    else return wc;
}

// Wavefront reductions: an xor butterfly over 32, 16, ..., 1 lanes of the
// 64-lane wave (cross-lane permutes, no LDS array, no barrier).  The pairing
// is fixed and a + b == b + a exactly, so every lane ends with the same
// value and the result is the same on every run.
template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

// Sum over a block of B = 64 k threads: wave sums, then the k wave results in
// wave order; every thread gets the result.  sh: k + 1 doubles of LDS.
template <int B>
__device__ inline double block_sum_waves(double v, double* sh)
{
    static_assert(B % 64 == 0, "whole waves");
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int k = 1; k < B / 64; k++) t += sh[k];
        sh[B / 64] = t;
    }
    __syncthreads();
    const double r = sh[B / 64];
    __syncthreads();   // sh may be reused by the caller
    return r;
}

// splitmix64 (Steele, Lea & Flood 2014): golden-gamma increment, then the
// published finaliser.
__host__ __device__ inline uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace lbm
