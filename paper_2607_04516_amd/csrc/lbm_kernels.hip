// HIP kernels of the D3Q19 LBM-LES update for gfx950 (arXiv 2607.04516,
// App. D): the fused in-place A-A collide-and-stream step, the out-of-place
// push step used to recompute trajectories, zero-gradient outflow passes,
// initialisation, state export/import, macroscopic fields, probes and
// reductions.
//
// In-place A-A streaming on the SoA array f[dir][z][y][x]:
//   even step  each cell reads its own 19 slots (natural layout: slot i of
//              cell x holds f_i(x)), collides, and writes f*_i back into
//              its own slot opp(i) (swapped layout);
//   odd step   each cell gathers f_i(x) = f*_i(x - c_i) from slot opp(i) of
//              the neighbour, collides, and scatters f*_i(x) into slot i of
//              cell x + c_i (natural layout again).
// Every slot is read and written by exactly one thread per step, so the
// update needs one array and no synchronisation.  The boundary rules enter
// only through the slot each direction resolves to (lbm_device.h).
#include "lbm_device.h"
#include "lbm_general.h"
#include "lbm_launch.h"

#include <type_traits>

namespace lbm {

// Wave -> (chunk, y, z) with a block order that keeps consecutive chunks of a
// row on one XCD (blocks are dealt to the 8 XCDs round robin).
__device__ inline long long xcd_block(long long nblocks_padded)
{
    const long long b = blockIdx.x;
    const long long per = nblocks_padded >> 3;
    return (b & 7) * per + (b >> 3);
}

// --------------------------------------------------------------------------
// Collide-and-stream step.
//   MODE_EVEN / MODE_ODD: in place on f (src == dst, padded layout).
//   MODE_PUSH: canonical src -> canonical dst (local read, scattered write).
// STATS: add u and u^2 of the pre-collision state into acc [6][N].
// --------------------------------------------------------------------------
template <int K, int MODE, bool STATS>
__global__ void __launch_bounds__(256)
k_step(typename Codec<K>::store* dst, const typename Codec<K>::store* src, const uint64_t* __restrict__ mask,
       const double* __restrict__ uin, const typename Codec<K>::store* __restrict__ ghost, Geo g, Lay ls, Lay ld,
       Phys<typename Codec<K>::real> P, typename Codec<K>::real* stats, long long nwaves, long long nblocks_padded,
       const unsigned* __restrict__ wlist)
{
    using C = Codec<K>;
    using R = typename C::real;
    const long long blk = xcd_block(nblocks_padded);
    long long wave = blk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    if (wlist) wave = wlist[wave];
    const int lane = threadIdx.x & 63;
    const int cx = (int)(wave % g.ncx);
    const long long row = wave / g.ncx;
    const int y = (int)(row % g.ny);
    const int z = (int)(row / g.ny);
    const int x = cx * 64 + lane;

    // ---------------- uniform fast-path test ----------------
    bool fast = (y >= 1) && (y <= g.ny - 2) && (z >= 1) && (z <= g.nz - 2) && (cx >= 1) && (cx * 64 + 63 <= g.nx - 2);
    if (fast) {
        uint64_t acc = 0;
#pragma unroll
        for (int dz = -1; dz <= 1; dz++)
#pragma unroll
            for (int dy = -1; dy <= 1; dy++) {
                const uint64_t* w = mask + (long long)((y + dy) + (long long)g.ny * (z + dz)) * g.wpr + cx;
                acc |= w[0] | (w[-1] >> 63) | (w[1] << 63);
            }
        fast = (acc == 0);
    }

    if (fast) {
        R h[NQ];
        static_for<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            constexpr V3 c = dirv(I);
            long long idx;
            if constexpr (MODE == MODE_ODD)
                idx = pop_index(ls, opp(I), x - c.x, y - c.y, z - c.z);
            else
                idx = pop_index(ls, I, x, y, z);
            h[I] = C::raw(src[idx]);
        });
        R drho, ux, uy, uz, tau;
        collide_at<R, C::SC>(h, P, g, x, y, z, drho, ux, uy, uz, tau);
        static_for<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            constexpr V3 c = dirv(I);
            long long idx;
            if constexpr (MODE == MODE_EVEN)
                idx = pop_index(ld, I, x, y, z);
            else
                idx = pop_index(ld, opp(I), x - c.x, y - c.y, z - c.z);
            dst[idx] = C::pack(h[opp(I)]);
        });
        if constexpr (STATS) {
            const long long n = x + (long long)g.nx * (y + (long long)g.ny * z);
            stats[n] += ux;
            stats[g.N + n] += uy;
            stats[2 * g.N + n] += uz;
            stats[3 * g.N + n] += ux * ux;
            stats[4 * g.N + n] += uy * uy;
            stats[5 * g.N + n] += uz * uz;
        }
        return;
    }

    // ---------------- general path: every boundary rule, per lane ----------------
    if (x >= g.nx) return;
    general_cell<K, MODE, STATS>(dst, src, mask, uin, ghost, g, ls, ld, P, stats, x, y, z);
}

// --------------------------------------------------------------------------
// Zero-gradient outflow passes over the outflow faces F.
//   ghost: before an odd step, store for each (cell on F, entering direction
//          owned by F) the value the inner cell q pulls (or the bounce-back
//          when q is solid), read from the swapped layout.  The odd step
//          reads these instead of slots its neighbours overwrite.
//   copy:  after an odd step (natural layout), or after a push step,
//          f_I(p) = f_I(q) for every such pair with q fluid.
// Every outflow face is a run of blocks of one launch.  The faces do not
// depend on each other: the ghost entries are per face, and with every
// extent >= 3 no copy source q lies on an outflow face through which its
// direction enters (q sits at 1 or n - 2 on each axis it was moved along,
// and on any other axis at the coordinate of p, which would have moved it),
// so no face reads a slot another face writes.  On the 800x800x128 grid
// (x+ and y+ outflow) one launch instead of one per face took the FP32
// ghost pass from 2 x 18 to 22 us and the copy from 2 x 22 to 38 us.
// --------------------------------------------------------------------------

// Cell t of face F (row-major over the face's two other axes).  Written
// with selects: assigning x, y, z under branches kept them in scratch.
__device__ inline bool face_cell(const Geo& g, int F, long long t, int& x, int& y, int& z)
{
    const int a = F >> 1;
    const int n0 = a == 0 ? g.ny : g.nx;
    const int n1 = a == 2 ? g.ny : g.nz;
    if (t >= (long long)n0 * n1) return false;
    const int u = (int)(t % n0), v = (int)(t / n0);
    const int w = (F & 1) ? (a == 0 ? g.nx : (a == 1 ? g.ny : g.nz)) - 1 : 0;
    x = a == 0 ? w : u;
    y = a == 0 ? u : (a == 1 ? w : v);
    z = a == 2 ? w : v;
    return true;
}

struct FaceRuns {
    int n;                 // outflow faces
    int face[6];           // their face indices
    long long first[7];    // first block of each face's run; first[n] = grid
    long long goff[6];     // their first ghost entries
};

// Face of this block and its cell index t; the runs are searched with
// constant indices (a runtime index into the by-value struct would put it
// in scratch memory).
__device__ inline int run_face(const FaceRuns& fr, long long& t, long long& goff)
{
    const long long b = blockIdx.x;
    int F = fr.face[0];
    long long start = 0;
    goff = fr.goff[0];
#pragma unroll
    for (int i = 1; i < 6; i++)
        if (i < fr.n && b >= fr.first[i]) { F = fr.face[i]; start = fr.first[i]; goff = fr.goff[i]; }
    t = (b - start) * (long long)blockDim.x + threadIdx.x;
    return F;
}

template <int K>
__global__ void __launch_bounds__(256)
k_outflow_ghost(const typename Codec<K>::store* f, const uint64_t* __restrict__ mask, typename Codec<K>::store* ghost,
                Geo g, Lay L, FaceRuns fr)
{
    int x, y, z;
    long long t, goff;
    const int F = run_face(fr, t, goff);
    if (!face_cell(g, F, t, x, y, z)) return;
    if (solid_at(mask, g, x, y, z) || inflow_face_of(g, x, y, z) >= 0) return;
    static_for<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        int qx, qy, qz, owner;
        if (!outflow_entering<I>(g, x, y, z, qx, qy, qz, owner) || owner != F) return;
        typename Codec<K>::store v;
        if (solid_at(mask, g, qx, qy, qz)) {
            v = f[pop_index(L, I, x, y, z)];
        } else {
            const Res r = resolve_plain<I>(g, mask, qx, qy, qz);
            v = f[pop_index(L, r.dir, r.x, r.y, r.z)];
        }
        ghost[ghost_index<I, true>(g, F, x, y, z, goff)] = v;
    });
}

template <int K>
__global__ void __launch_bounds__(256)
k_outflow_copy(typename Codec<K>::store* f, const uint64_t* __restrict__ mask, Geo g, Lay L, FaceRuns fr)
{
    int x, y, z;
    long long t, goff;
    const int F = run_face(fr, t, goff);
    if (!face_cell(g, F, t, x, y, z)) return;
    if (solid_at(mask, g, x, y, z) || inflow_face_of(g, x, y, z) >= 0) return;
    static_for<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        int qx, qy, qz, owner;
        if (!outflow_entering<I>(g, x, y, z, qx, qy, qz, owner) || owner != F) return;
        if (solid_at(mask, g, qx, qy, qz)) return;
        f[pop_index(L, I, x, y, z)] = f[pop_index(L, I, qx, qy, qz)];
    });
}

// --------------------------------------------------------------------------
// Populations of one cell in the current state (phase 0: natural layout,
// phase 1: swapped layout after an even step, resolved through the full
// streaming rules).  Cell must be fluid and not an inflow cell.
// --------------------------------------------------------------------------
template <int K>
__device__ inline void load_cell(const typename Codec<K>::store* f, const uint64_t* __restrict__ mask, const Geo& g,
                                 const Lay& L, int phase, int x, int y, int z, typename Codec<K>::store* out)
{
    static_for<0, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if (phase == 0) {
            out[I] = f[pop_index(L, I, x, y, z)];
        } else {
            const Res r = resolve_full<I>(g, mask, x, y, z);
            out[I] = f[pop_index(L, r.dir, r.x, r.y, r.z)];
        }
    });
}

// Initial state: feq(rho0, u0(z) + noise) in fluid cells (double precision,
// then encoded), 0 in solid cells and padding.
template <int K>
__global__ void __launch_bounds__(256)
k_init(typename Codec<K>::store* f, const uint64_t* __restrict__ mask, const double* __restrict__ uin,
       const double* __restrict__ u0, Geo g, Lay L, double rho0, double amp, uint64_t seed)
{
    using C = Codec<K>;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long cells = (long long)L.pitch * g.ny * g.nz;
    if (t >= cells) return;
    const int x = (int)(t % L.pitch);
    const long long row = t / L.pitch;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    double h[NQ];
    for (int i = 0; i < NQ; i++) h[i] = 0.0;
    if (x < g.nx && !solid_at(mask, g, x, y, z)) {
        double u[3];
        const int inf = inflow_face_of(g, x, y, z);
        if (inf >= 0) {
            load_inflow<double>(uin, g, inf, x, y, z, u[0], u[1], u[2]);
        } else {
            const long long n = x + (long long)g.nx * (y + (long long)g.ny * z);
            for (int c = 0; c < 3; c++) {
                const uint64_t r = splitmix64(seed + 3ull * (uint64_t)n + (uint64_t)c);
                const double unit = (double)(r >> 11) * (1.0 / 9007199254740992.0);
                u[c] = u0[3 * z + c] + amp * (2.0 * unit - 1.0);
            }
        }
        equilibrium_shifted<double>(rho0, 0.0, u[0], u[1], u[2], h);
    }
    for (int i = 0; i < NQ; i++) f[pop_index(L, i, x, y, z)] = C::enc((typename C::real)h[i]);
}

// Canonical export: dst[i][n] = h_i(x, t) (unpadded), inflow cells at their
// equilibrium, solid cells 0.
template <int K>
__global__ void __launch_bounds__(256)
k_export(const typename Codec<K>::store* f, const uint64_t* __restrict__ mask, const double* __restrict__ uin,
         Geo g, Lay L, Phys<typename Codec<K>::real> P, int phase, typename Codec<K>::store* dst)
{
    using C = Codec<K>;
    using R = typename C::real;
    const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx);
    const long long row = n / g.nx;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    typename C::store v[NQ];
    if (solid_at(mask, g, x, y, z)) {
        for (int i = 0; i < NQ; i++) v[i] = C::enc(R(0));
    } else {
        const int inf = inflow_face_of(g, x, y, z);
        if (inf >= 0) {
            R u[3], heq[NQ];
            load_inflow<R>(uin, g, inf, x, y, z, u[0], u[1], u[2]);
            equilibrium_shifted<R>(P.rho0, R(0), u[0], u[1], u[2], heq);
            for (int i = 0; i < NQ; i++) v[i] = C::enc(heq[i]);
        } else {
            load_cell<K>(f, mask, g, L, phase, x, y, z, v);
        }
    }
    for (int i = 0; i < NQ; i++) dst[(long long)i * g.N + n] = v[i];
}

// Canonical import into the natural layout (phase 0).
template <int K>
__global__ void __launch_bounds__(256)
k_import(typename Codec<K>::store* f, const uint64_t* __restrict__ mask, Geo g, Lay L,
         const typename Codec<K>::store* src)
{
    using C = Codec<K>;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long cells = (long long)L.pitch * g.ny * g.nz;
    if (t >= cells) return;
    const int x = (int)(t % L.pitch);
    const long long row = t / L.pitch;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    const bool live = x < g.nx && !solid_at(mask, g, x, y, z) && inflow_face_of(g, x, y, z) < 0;
    const long long n = x + (long long)g.nx * row;
    for (int i = 0; i < NQ; i++)
        f[pop_index(L, i, x, y, z)] = live ? src[(long long)i * g.N + n] : C::enc(typename C::real(0));
}

// Macroscopic fields (rho, u, nu_t = (tau_eff - tau0)/3) of the current state.
template <int K>
__global__ void __launch_bounds__(256)
k_macros(const typename Codec<K>::store* f, const uint64_t* __restrict__ mask, const double* __restrict__ uin,
         Geo g, Lay L, Phys<typename Codec<K>::real> P, int phase, typename Codec<K>::real* rho,
         typename Codec<K>::real* u, typename Codec<K>::real* nut)
{
    using C = Codec<K>;
    using R = typename C::real;
    const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx);
    const long long row = n / g.nx;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    R r = P.rho0, ux = 0, uy = 0, uz = 0, nt = 0;
    if (!solid_at(mask, g, x, y, z)) {
        const int inf = inflow_face_of(g, x, y, z);
        if (inf >= 0) {
            load_inflow<R>(uin, g, inf, x, y, z, ux, uy, uz);
        } else {
            typename C::store v[NQ];
            load_cell<K>(f, mask, g, L, phase, x, y, z, v);
            R h[NQ];
            for (int i = 0; i < NQ; i++) h[i] = C::dec(v[i]);
            R drho, tau;
            collide_pairs<R, 1>(h, P, drho, ux, uy, uz, tau);
            r = P.rho0 + drho;
            nt = (tau - P.tau0) / R(3);
        }
    }
    if (rho) rho[n] = r;
    if (u) {
        u[n] = ux;
        u[g.N + n] = uy;
        u[2 * g.N + n] = uz;
    }
    if (nut) nut[n] = nt;
}

// rho and u of one cell for probes (solid: rho0, 0; inflow: rho0, u_in).
template <int K>
__device__ inline void cell_rho_u(const typename Codec<K>::store* f, const uint64_t* __restrict__ mask,
                                  const double* __restrict__ uin, const Geo& g, const Lay& L,
                                  const Phys<typename Codec<K>::real>& P, int phase, int x, int y, int z,
                                  typename Codec<K>::real* out)
{
    using C = Codec<K>;
    using R = typename C::real;
    out[0] = P.rho0;
    out[1] = out[2] = out[3] = R(0);
    if (solid_at(mask, g, x, y, z)) return;
    const int inf = inflow_face_of(g, x, y, z);
    if (inf >= 0) {
        load_inflow<R>(uin, g, inf, x, y, z, out[1], out[2], out[3]);
        return;
    }
    typename C::store v[NQ];
    load_cell<K>(f, mask, g, L, phase, x, y, z, v);
    R h[NQ];
    for (int i = 0; i < NQ; i++) h[i] = C::dec(v[i]);
    R drho;
    moments_pairs<R, 1>(h, P, drho, out[1], out[2], out[3]);
    out[0] = P.rho0 + drho;
}

template <int K>
__global__ void k_probe_points(const typename Codec<K>::store* f, const uint64_t* __restrict__ mask,
                               const double* __restrict__ uin, Geo g, Lay L, Phys<typename Codec<K>::real> P,
                               int phase, const float* pts, int np, float* out)
{
    using R = typename Codec<K>::real;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    float c[3] = {pts[3 * p], pts[3 * p + 1], pts[3 * p + 2]};
    const int n[3] = {g.nx, g.ny, g.nz};
    int i0[3];
    float fr[3];
    for (int a = 0; a < 3; a++) {
        float v = fminf(fmaxf(c[a], 0.0f), float(n[a] - 1));
        int b = (int)floorf(v);
        if (b > n[a] - 1) b = n[a] - 1;
        i0[a] = b;
        fr[a] = v - float(b);
    }
    R acc[4] = {0, 0, 0, 0};
    for (int k = 0; k < 8; k++) {
        const int d[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
        R w = 1;
        int q[3];
        for (int a = 0; a < 3; a++) {
            w *= d[a] ? R(fr[a]) : R(1) - R(fr[a]);
            q[a] = min(i0[a] + d[a], n[a] - 1);
        }
        if (w == R(0)) continue;
        R v[4];
        cell_rho_u<K>(f, mask, uin, g, L, P, phase, q[0], q[1], q[2], v);
        for (int j = 0; j < 4; j++) acc[j] += w * v[j];
    }
    for (int j = 0; j < 4; j++) out[4 * p + j] = float(acc[j]);
}

template <int K>
__global__ void k_probe_cells(const typename Codec<K>::store* f, const uint64_t* __restrict__ mask,
                              const double* __restrict__ uin, Geo g, Lay L, Phys<typename Codec<K>::real> P,
                              int phase, const int* cells, int np, typename Codec<K>::real* acc)
{
    using R = typename Codec<K>::real;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    R v[4];
    cell_rho_u<K>(f, mask, uin, g, L, P, phase, cells[3 * p], cells[3 * p + 1], cells[3 * p + 2], v);
    // Neumaier summation: acc[0][p] holds the running sum, acc[1][p] the
    // accumulated rounding errors of its additions
    R* sum = acc + 3 * p;
    R* cmp = acc + 3 * (long long)np + 3 * p;
    for (int a = 0; a < 3; a++) {
        const R s = sum[a], x = v[1 + a];
        const R t = s + x;
        cmp[a] += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
        sum[a] = t;
    }
}

// --------------------------------------------------------------------------
// Mass / energy / watchdog reduction over fluid, non-inflow cells.
// Pass 1: per lane a Neumaier-compensated sum of rho - rho0 in the real
// type and double sums of the kinetic energy, plus max |u|^2, max |rho-rho0|
// and a non-finite flag; then wavefront reductions (xor butterflies) and the
// block's four wave results in order, all in double.
// Pass 2: one block reduces the block partials in a fixed order.
// --------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

template <int K>
__global__ void __launch_bounds__(RED_THREADS)
k_mass_partial(const typename Codec<K>::store* f, const uint64_t* __restrict__ mask, Geo g, Lay L,
               Phys<typename Codec<K>::real> P, int phase, double* partial)
{
    using C = Codec<K>;
    using R = typename C::real;
    R s = 0, comp = 0;
    double e = 0, umax = 0, dmax = 0, bad = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < g.N; n += stride) {
        const int x = (int)(n % g.nx);
        const long long row = n / g.nx;
        const int y = (int)(row % g.ny), z = (int)(row / g.ny);
        if (solid_at(mask, g, x, y, z) || inflow_face_of(g, x, y, z) >= 0) continue;
        typename C::store v[NQ];
        load_cell<K>(f, mask, g, L, phase, x, y, z, v);
        R h[NQ];
        for (int i = 0; i < NQ; i++) h[i] = C::dec(v[i]);
        R drho, ux, uy, uz;
        moments_pairs<R, 1>(h, P, drho, ux, uy, uz);
        // Neumaier summation of drho
        const R tsum = s + drho;
        if (fabs((double)s) >= fabs((double)drho)) comp += (s - tsum) + drho;
        else comp += (drho - tsum) + s;
        s = tsum;
        const double rho = (double)P.rho0 + (double)drho;
        const double u2 = (double)ux * ux + (double)uy * uy + (double)uz * uz;
        e += 0.5 * rho * u2;
        if (!(u2 <= 1e300) || !(fabs((double)drho) <= 1e300)) bad = 1;
        umax = fmax(umax, u2);
        dmax = fmax(dmax, fabs((double)drho));
    }
    // wavefront reductions, then the block's waves in order
    constexpr int NW = RED_THREADS / 64;
    __shared__ double sh[5][NW];
    const double r[5] = {wave_sum((double)s + (double)comp), wave_sum(e), wave_max(umax), wave_max(dmax),
                         wave_max(bad)};
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 5; k++) sh[k][threadIdx.x >> 6] = r[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double a[5] = {sh[0][0], sh[1][0], sh[2][0], sh[3][0], sh[4][0]};
        for (int w = 1; w < NW; w++) {
            a[0] += sh[0][w];
            a[1] += sh[1][w];
            for (int k = 2; k < 5; k++) a[k] = fmax(a[k], sh[k][w]);
        }
        for (int k = 0; k < 5; k++) partial[5 * blockIdx.x + k] = a[k];
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_mass_final(const double* partial, int nb, double* out)
{
    __shared__ double sh[5][RED_THREADS / 64];
    double a[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += RED_THREADS) {
        a[0] += partial[5 * b];
        a[1] += partial[5 * b + 1];
        a[2] = fmax(a[2], partial[5 * b + 2]);
        a[3] = fmax(a[3], partial[5 * b + 3]);
        a[4] = fmax(a[4], partial[5 * b + 4]);
    }
    const double r[5] = {wave_sum(a[0]), wave_sum(a[1]), wave_max(a[2]), wave_max(a[3]), wave_max(a[4])};
    constexpr int NW = RED_THREADS / 64;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 5; k++) sh[k][threadIdx.x >> 6] = r[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[5] = {sh[0][0], sh[1][0], sh[2][0], sh[3][0], sh[4][0]};
        for (int w = 1; w < NW; w++) {
            t[0] += sh[0][w];
            t[1] += sh[1][w];
            for (int k = 2; k < 5; k++) t[k] = fmax(t[k], sh[k][w]);
        }
        for (int k = 0; k < 5; k++) out[k] = t[k];
    }
}

// Wave-mask table, built once per grid: the solid-source masks of every wave
// (one 64-cell chunk of a row) that has a solid neighbour, so the fast
// kernels read 18 words instead of rebuilding them from the mask rows.
__global__ void __launch_bounds__(256)
k_wave_masks(const uint64_t* __restrict__ mask, Geo g, int* idx, uint64_t* tab, long long nwaves, int pass)
{
    const long long wave = blockIdx.x * 4ll + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int lane = threadIdx.x & 63;
    const int cx = (int)(wave % g.ncx);
    const long long row = wave / g.ncx;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    RowWin W;
    load_rows(W, mask, g, cx, y, z);
    if (pass == 0) {
        uint64_t any = 0;
        static_for<1, NQ>([&](auto ic) { any |= solid_src_mask<decltype(ic)::value>(W); });
        if (lane == 0) idx[wave] = any != 0 ? 1 : 0;
        return;
    }
    const int k = idx[wave];
    if (k < 0) return;
    static_for<1, NQ>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if (lane == I - 1) tab[18ll * k + (I - 1)] = solid_src_mask<I>(W);
    });
}

hipError_t launch_wave_masks(const DevCtx& d, int* idx, uint64_t* tab, int pass, hipStream_t s)
{
    const long long nwaves = (long long)d.g.ncx * d.g.ny * d.g.nz;
    hipLaunchKernelGGL(k_wave_masks, dim3((unsigned)((nwaves + 3) / 4)), dim3(256), 0, s, d.mask, d.g, idx, tab,
                       nwaves, pass);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Host launchers
// --------------------------------------------------------------------------

static inline unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// General odd-step kernel over the listed waves (rows on a y or z face, x
// faces other than inflow at x- / outflow at x+).
template <int K, bool ST>
static hipError_t general_odd_k(const DevCtx& d, void* stats, hipStream_t s)
{
    using C = Codec<K>;
    const long long nwaves = d.odd_list_n;
    if (nwaves == 0) return hipSuccess;
    const long long nb = (nwaves + 3) / 4;
    const long long nbp = (nb + 7) / 8 * 8;
    const Lay L{d.g.S, d.g.pitch, d.g.lrb, d.g.nyp};
    hipLaunchKernelGGL((k_step<K, MODE_ODD, ST>), dim3((unsigned)nbp), dim3(256), 0, s, (typename C::store*)d.f,
                       (const typename C::store*)d.f, d.mask, d.uin, (const typename C::store*)d.ghost, d.g, L, L,
                       phys_of<K>(d), (typename C::real*)stats, nwaves, nbp, d.odd_list);
    return hipGetLastError();
}

#define LBM_DISPATCH(codec, ...)                      \
    switch (codec) {                                  \
        case 0: { constexpr int K = 0; __VA_ARGS__; } \
        case 1: { constexpr int K = 1; __VA_ARGS__; } \
        case 2: { constexpr int K = 2; __VA_ARGS__; } \
        case 3: { constexpr int K = 3; __VA_ARGS__; } \
        default: return hipErrorInvalidValue;         \
    }

static Lay padded(const DevCtx& d) { return Lay{d.g.S, d.g.pitch, d.g.lrb, d.g.nyp}; }
static Lay canonical(const DevCtx& d) { return Lay{d.g.N, d.g.nx, -1, d.g.ny}; }

hipError_t launch_general_odd(const DevCtx& d, void* stats, hipStream_t s)
{
    LBM_DISPATCH(d.codec, {
        if (stats) return general_odd_k<K, true>(d, stats, s);
        return general_odd_k<K, false>(d, stats, s);
    });
}

static long long face_cells(const Geo& g, int F)
{
    const int a = F >> 1;
    return a == 0 ? (long long)g.ny * g.nz : (a == 1 ? (long long)g.nx * g.nz : (long long)g.nx * g.ny);
}

static FaceRuns outflow_runs(const Geo& g)
{
    FaceRuns fr{};
    long long b = 0;
    for (int F = 0; F < 6; F++) {
        if (g.face[F] != F_OUTFLOW) continue;
        fr.face[fr.n] = F;
        fr.first[fr.n] = b;
        fr.goff[fr.n] = g.ghost_off[F];
        b += blocks_for(face_cells(g, F), 256);
        fr.n++;
    }
    fr.first[fr.n] = b;
    return fr;
}

hipError_t launch_outflow_ghost(const DevCtx& d, hipStream_t s)
{
    const FaceRuns fr = outflow_runs(d.g);
    if (fr.n == 0) return hipSuccess;
    LBM_DISPATCH(d.codec, {
        hipLaunchKernelGGL((k_outflow_ghost<K>), dim3((unsigned)fr.first[fr.n]), dim3(256), 0, s,
                           (const typename Codec<K>::store*)d.f, d.mask, (typename Codec<K>::store*)d.ghost, d.g,
                           padded(d), fr);
        break;
    });
    return hipGetLastError();
}

hipError_t launch_outflow_copy(const DevCtx& d, void* arr, int canonical_layout, hipStream_t s)
{
    const Lay L = canonical_layout ? canonical(d) : padded(d);
    const FaceRuns fr = outflow_runs(d.g);
    if (fr.n == 0) return hipSuccess;
    LBM_DISPATCH(d.codec, {
        hipLaunchKernelGGL((k_outflow_copy<K>), dim3((unsigned)fr.first[fr.n]), dim3(256), 0, s,
                           (typename Codec<K>::store*)arr, d.mask, d.g, L, fr);
        break;
    });
    return hipGetLastError();
}

hipError_t launch_init(const DevCtx& d, const double* u0_dev, double amp, uint64_t seed, hipStream_t s)
{
    const long long cells = (long long)d.g.pitch * d.g.ny * d.g.nz;
    LBM_DISPATCH(d.codec, {
        hipLaunchKernelGGL((k_init<K>), dim3(blocks_for(cells, 256)), dim3(256), 0, s, (typename Codec<K>::store*)d.f,
                           d.mask, d.uin, u0_dev, d.g, padded(d), d.rho0, amp, seed);
        return hipGetLastError();
    });
}

hipError_t launch_export(const DevCtx& d, int phase, void* dst, hipStream_t s)
{
    LBM_DISPATCH(d.codec, {
        hipLaunchKernelGGL((k_export<K>), dim3(blocks_for(d.g.N, 256)), dim3(256), 0, s,
                           (const typename Codec<K>::store*)d.f, d.mask, d.uin, d.g, padded(d), phys_of<K>(d), phase,
                           (typename Codec<K>::store*)dst);
        return hipGetLastError();
    });
}

hipError_t launch_import(const DevCtx& d, const void* src, hipStream_t s)
{
    const long long cells = (long long)d.g.pitch * d.g.ny * d.g.nz;
    LBM_DISPATCH(d.codec, {
        hipLaunchKernelGGL((k_import<K>), dim3(blocks_for(cells, 256)), dim3(256), 0, s,
                           (typename Codec<K>::store*)d.f, d.mask, d.g, padded(d), (const typename Codec<K>::store*)src);
        return hipGetLastError();
    });
}

hipError_t launch_macros(const DevCtx& d, int phase, void* rho, void* u, void* nut, hipStream_t s)
{
    LBM_DISPATCH(d.codec, {
        using R = typename Codec<K>::real;
        hipLaunchKernelGGL((k_macros<K>), dim3(blocks_for(d.g.N, 256)), dim3(256), 0, s,
                           (const typename Codec<K>::store*)d.f, d.mask, d.uin, d.g, padded(d), phys_of<K>(d), phase,
                           (R*)rho, (R*)u, (R*)nut);
        return hipGetLastError();
    });
}

hipError_t launch_probe_points(const DevCtx& d, int phase, const float* pts, int np, float* out, hipStream_t s)
{
    LBM_DISPATCH(d.codec, {
        hipLaunchKernelGGL((k_probe_points<K>), dim3(blocks_for(np, 64)), dim3(64), 0, s,
                           (const typename Codec<K>::store*)d.f, d.mask, d.uin, d.g, padded(d), phys_of<K>(d), phase,
                           pts, np, out);
        return hipGetLastError();
    });
}

hipError_t launch_probe_cells(const DevCtx& d, int phase, const int* cells, int np, void* acc, hipStream_t s)
{
    LBM_DISPATCH(d.codec, {
        using R = typename Codec<K>::real;
        hipLaunchKernelGGL((k_probe_cells<K>), dim3(blocks_for(np, 64)), dim3(64), 0, s,
                           (const typename Codec<K>::store*)d.f, d.mask, d.uin, d.g, padded(d), phys_of<K>(d), phase,
                           cells, np, (R*)acc);
        return hipGetLastError();
    });
}

int mass_blocks(const Geo& g)
{
    long long nb = (g.N + RED_THREADS - 1) / RED_THREADS;
    return (int)(nb < 2048 ? nb : 2048);
}

hipError_t launch_mass(const DevCtx& d, int phase, double* partial, double* out5, hipStream_t s)
{
    const int nb = mass_blocks(d.g);
    LBM_DISPATCH(d.codec, {
        hipLaunchKernelGGL((k_mass_partial<K>), dim3(nb), dim3(RED_THREADS), 0, s,
                           (const typename Codec<K>::store*)d.f, d.mask, d.g, padded(d), phys_of<K>(d), phase, partial);
        hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(RED_THREADS), 0, s, partial, nb, out5);
        return hipGetLastError();
    });
}

}  // namespace lbm
