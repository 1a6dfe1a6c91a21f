// Discrete adjoint of the D3Q19 LBM-LES step for gfx950.
//
// The forward step is f(t+1) = S(C(f(t)), u_in): C the local collision of
// App. D (eqs. D.1-D.4, D.8, D.10, D.11, Guo source), S the streaming with
// its boundary rules, inflow cells supplying feq(rho0, u_in).  One adjoint
// step computes
//   lam(t) = J_C(f(t))^T S^T lam(t+1)            (+ probe sources)
//   g[face][z] += sum over the face's inflow cells of lam*_k d feq_k/du_in
// on canonical unpadded arrays:
//   * S^T is a gather: the post-collision population k of cell x lands in
//     the slot that the pull of direction opp(k) at x resolves to (the same
//     slot the forward scatter writes), plus every zero-gradient outflow
//     copy of that slot (up to 7 at an outflow corner);
//   * J_C^T is applied matrix-free from the hand-derived derivatives of the
//     moments, the equilibrium, the invariant Q and tau_eff.
// Solid and inflow cells get lam = 0 (their state is not a variable).
#include "lbm_device.h"
#include "lbm_launch.h"

#include <type_traits>

namespace lbm {

template <int I, int N, class Fn>
__device__ __forceinline__ void adj_static_for(Fn&& fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        adj_static_for<I + 1, N>(fn);
    }
}

__device__ inline long long cidx(const Geo& g, int x, int y, int z)
{
    return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

// Sum of lam_next over the zero-gradient outflow copies of slot (d, m):
// every outflow cell c whose entering population m copies what d receives.
template <typename R>
__device__ inline R copy_partner_sum(const R* lam_next, const uint64_t* __restrict__ mask, const Geo& g, int dx,
                                     int dy, int dz, int m, int vx, int vy, int vz)
{
    // per axis: the side (+1 high, -1 low) of an outflow face that m enters
    // and d lies next to, or 0
    int sx = 0, sy = 0, sz = 0;
    if (vx == -1 && g.face[1] == F_OUTFLOW && dx == g.nx - 2) sx = 1;
    else if (vx == 1 && g.face[0] == F_OUTFLOW && dx == 1) sx = -1;
    if (vy == -1 && g.face[3] == F_OUTFLOW && dy == g.ny - 2) sy = 1;
    else if (vy == 1 && g.face[2] == F_OUTFLOW && dy == 1) sy = -1;
    if (vz == -1 && g.face[5] == F_OUTFLOW && dz == g.nz - 2) sz = 1;
    else if (vz == 1 && g.face[4] == F_OUTFLOW && dz == 1) sz = -1;
    R s = R(0);
    if ((sx | sy | sz) == 0) return s;
    // every non-empty subset of those axes moves d onto one copy cell
    for (int sub = 1; sub < 8; sub++) {
        if (((sub & 1) && !sx) || ((sub & 2) && !sy) || ((sub & 4) && !sz)) continue;
        const int cx = dx + ((sub & 1) ? sx : 0);
        const int cy = dy + ((sub & 2) ? sy : 0);
        const int cz = dz + ((sub & 4) ? sz : 0);
        if (!solid_at(mask, g, cx, cy, cz) && inflow_face_of(g, cx, cy, cz) < 0)
            s += lam_next[(long long)m * g.N + cidx(g, cx, cy, cz)];
    }
    return s;
}

// lam* of post-collision population opp(I) of cell (x,y,z): lam_next at
// every slot that value is streamed into.  INFLOW: the cell is an inflow
// cell (its forward scatter has no outflow rule and its own slots are void).
template <typename R, int I, bool INFLOW>
__device__ inline R adj_gather(const R* lam_next, const uint64_t* __restrict__ mask, const Geo& g, int x, int y, int z)
{
    if constexpr (!INFLOW) {
        int qx, qy, qz, owner;
        if (outflow_entering<I>(g, x, y, z, qx, qy, qz, owner)) {
            // opp(I) leaves through an outflow face: only the bounce-back of a
            // solid inner neighbour keeps it, in the cell's own slot I
            // (x, I) is itself an outflow copy slot: nothing copies from it
            if (!solid_at(mask, g, qx, qy, qz)) return R(0);
            return lam_next[(long long)I * g.N + cidx(g, x, y, z)];
        }
    }
    const Res r = resolve_plain<I>(g, mask, x, y, z);
    if (r.kind != 0) return R(0);
    if (inflow_face_of(g, r.x, r.y, r.z) >= 0) return R(0);
    if constexpr (INFLOW) {
        if (r.x == x && r.y == y && r.z == z) return R(0);
    }
    return lam_next[(long long)r.dir * g.N + cidx(g, r.x, r.y, r.z)] +
           copy_partner_sum<R>(lam_next, mask, g, r.x, r.y, r.z, r.dir, r.vx, r.vy, r.vz);
}

// mu = J_C(h)^T ls for one cell (h shifted populations, in place into ls).
//
// Every sum over directions that the transpose needs is a low moment of the
// adjoint populations: with the pair sums a_k = ls_+ + ls_- and differences
// b_k = ls_+ - ls_- of the nine opposite pairs, the weighted moments
// S0 = sum w ls, S_a = sum w ls c_a and S_ab = sum w ls c_a c_b give
//   A   = sum ls feq / rho = S0 (1 - 3/2 u.u) + 3 S.u + 9/2 u.S2.u,
//   V_a = rho (3 S_a + 9 (S2 u)_a - 3 u_a S0)        (feq's u-derivative),
//   E_a = -3 F_a S0 + 9 (S2 F)_a,  P = 3 S.F - 3 u.F S0 + 9 u.S2.F  (Guo),
// and G = sum ls (h - heq) = sum ls h - rho A + rho0 S0.  Pi comes from the
// second moment of h as in the forward collision.  The result per pair is
// an even part (shared) plus or minus an odd part.
template <typename R>
__device__ inline void collision_transpose(const R* h, R* ls, const Phys<R>& P)
{
    R drho, ux, uy, uz, Fx, Fy, Fz;
    moments_pairs<R, 1>(h, P, drho, ux, uy, uz, Fx, Fy, Fz);
    const R rho = P.rho0 + drho;
    const R inv_rho = R(1) / rho;
    // non-equilibrium second moment Pi = M - drho/3 I - rho u u
    const R s1 = h[1] + h[2], s2 = h[3] + h[4], s3 = h[5] + h[6], s4 = h[7] + h[8], s5 = h[9] + h[10];
    const R s6 = h[11] + h[12], s7 = h[13] + h[14], s8 = h[15] + h[16], s9 = h[17] + h[18];
    const R t3 = drho * R(1.0 / 3.0);
    const R pxx = (((s1 + s4) + (s5 + s7)) + s8) - t3 - rho * ux * ux;
    const R pyy = (((s2 + s4) + (s6 + s7)) + s9) - t3 - rho * uy * uy;
    const R pzz = (((s3 + s5) + (s6 + s8)) + s9) - t3 - rho * uz * uz;
    const R pxy = (s4 - s7) - rho * ux * uy;
    const R pxz = (s5 - s8) - rho * ux * uz;
    const R pyz = (s6 - s9) - rho * uy * uz;
    const R pp = (pxx * pxx + pyy * pyy + pzz * pzz) + R(2) * (pxy * pxy + pxz * pxz + pyz * pyz);
    const R q = sqrt(R(2) * pp);
    const R D = P.tau0 * P.tau0 + P.ksmag * q * inv_rho;
    const R sD = sqrt(D);
    const R tau = R(0.5) * (P.tau0 + sD);
    const R omega = R(1) / tau;

    // moments of the adjoint populations
    constexpr R w0 = R(1.0 / 3.0), wf = R(1.0 / 18.0), we = R(1.0 / 36.0);
    R a[10], b[10];
#pragma unroll
    for (int k = 1; k <= 9; k++) {
        a[k] = ls[2 * k - 1] + ls[2 * k];
        b[k] = ls[2 * k - 1] - ls[2 * k];
    }
    R Lh = ls[0] * h[0];
#pragma unroll
    for (int i = 1; i < NQ; i++) Lh += ls[i] * h[i];
    const R S0 = w0 * ls[0] + wf * ((a[1] + a[2]) + a[3]) + we * (((a[4] + a[5]) + (a[6] + a[7])) + (a[8] + a[9]));
    const R Sx = wf * b[1] + we * ((b[4] + b[5]) + (b[7] + b[8]));
    const R Sy = wf * b[2] + we * ((b[4] + b[6]) + (b[9] - b[7]));
    const R Sz = wf * b[3] + we * ((b[5] + b[6]) - (b[8] + b[9]));
    const R Sxx = wf * a[1] + we * ((a[4] + a[5]) + (a[7] + a[8]));
    const R Syy = wf * a[2] + we * ((a[4] + a[6]) + (a[7] + a[9]));
    const R Szz = wf * a[3] + we * ((a[5] + a[6]) + (a[8] + a[9]));
    const R Sxy = we * (a[4] - a[7]), Sxz = we * (a[5] - a[8]), Syz = we * (a[6] - a[9]);
    // S2 u and S2 F
    const R tx = Sxx * ux + Sxy * uy + Sxz * uz;
    const R ty = Sxy * ux + Syy * uy + Syz * uz;
    const R tz = Sxz * ux + Syz * uy + Szz * uz;
    const R usq = ux * ux + uy * uy + uz * uz;
    const R A = S0 * (R(1) - R(1.5) * usq) + R(3) * (Sx * ux + Sy * uy + Sz * uz) +
                R(4.5) * (ux * tx + uy * ty + uz * tz);
    const R G = Lh - rho * A + P.rho0 * S0;
    const R vx = rho * (R(3) * Sx + R(9) * tx - R(3) * ux * S0);
    const R vy = rho * (R(3) * Sy + R(9) * ty - R(3) * uy * S0);
    const R vz = rho * (R(3) * Sz + R(9) * tz - R(3) * uz * S0);
    R Wx = omega * vx, Wy = omega * vy, Wz = omega * vz;
    R Pw = R(0);
    if (P.has_force) {
        const R ex = Sxx * Fx + Sxy * Fy + Sxz * Fz;
        const R ey = Sxy * Fx + Syy * Fy + Syz * Fz;
        const R ez = Sxz * Fx + Syz * Fy + Szz * Fz;
        const R uF = ux * Fx + uy * Fy + uz * Fz;
        Pw = R(3) * (Sx * Fx + Sy * Fy + Sz * Fz) - R(3) * uF * S0 + R(9) * (ux * ex + uy * ey + uz * ez);
        const R pre = R(1) - R(0.5) * omega;
        Wx += pre * (R(-3) * Fx * S0 + R(9) * ex);
        Wy += pre * (R(-3) * Fy * S0 + R(9) * ey);
        Wz += pre * (R(-3) * Fz * S0 + R(9) * ez);
    }
    Wx *= inv_rho;
    Wy *= inv_rho;
    Wz *= inv_rho;
    const R Wu = Wx * ux + Wy * uy + Wz * uz;
    // Coriolis: F = F0 - W2 x m, so d F / d f_j = D c_j with D v = -W2 x v,
    // and rho du/df_j = M c_j - u with M = I + D/2.  The c_j-linear part of
    // mu becomes c_j . (M^T W + (1 - omega/2) D^T V / rho), and D^T = -D
    // (D is antisymmetric): M^T v = v + (W2 x v)/2, D^T v = W2 x v.
    const R* W2 = P.W2;
    if (P.has_rot) {
        const R pre = (R(1) - R(0.5) * omega) * inv_rho;
        const R ax = Wx + R(0.5) * (W2[1] * Wz - W2[2] * Wy) + pre * (W2[1] * vz - W2[2] * vy);
        const R ay = Wy + R(0.5) * (W2[2] * Wx - W2[0] * Wz) + pre * (W2[2] * vx - W2[0] * vz);
        const R az = Wz + R(0.5) * (W2[0] * Wy - W2[1] * Wx) + pre * (W2[0] * vy - W2[1] * vx);
        Wx = ax;
        Wy = ay;
        Wz = az;
    }
    // closure: -(d omega/d f_j)(G + P/2) = Z (dQ_j - Q/rho),
    // dQ_j = (2/Q)[c.Pi.c - 2 (M c).Pi u + u.Pi.u - tr(Pi)/3]
    R Zt = R(0), base = R(0), Zq = R(0);
    R pux = 0, puy = 0, puz = 0;
    if (P.ksmag > R(0) && q > R(0)) {
        const R Z = (G + R(0.5) * Pw) * omega * omega * P.ksmag / (R(4) * sD) * inv_rho;
        Zt = Z * (R(2) / q);
        Zq = Z * q * inv_rho;
        pux = pxx * ux + pxy * uy + pxz * uz;
        puy = pxy * ux + pyy * uy + pyz * uz;
        puz = pxz * ux + pyz * uy + pzz * uz;
        base = (ux * pux + uy * puy + uz * puz) - (pxx + pyy + pzz) / R(3);
        if (P.has_rot) {   // (M c).Pi u = c . M^T (Pi u)
            const R ax = pux + R(0.5) * (W2[1] * puz - W2[2] * puy);
            const R ay = puy + R(0.5) * (W2[2] * pux - W2[0] * puz);
            const R az = puz + R(0.5) * (W2[0] * puy - W2[1] * pux);
            pux = ax;
            puy = ay;
            puz = az;
        }
    }
    const R om1 = R(1) - omega;
    const R e0 = omega * A - Wu + Zt * base - Zq;   // the c-independent part of every mu_j
    ls[0] = om1 * ls[0] + e0;
    // pair k (directions 2k-1 = +c and 2k = -c): mu = om1 ls + even +- odd
#define LBM_ADJ_PAIR(k, cpc, cw, cpu)                          \
    {                                                          \
        const R ev = e0 + Zt * (cpc);                          \
        const R od = (cw) - R(2) * Zt * (cpu);                 \
        ls[2 * (k) - 1] = om1 * ls[2 * (k) - 1] + (ev + od);   \
        ls[2 * (k)] = om1 * ls[2 * (k)] + (ev - od);           \
    }
    LBM_ADJ_PAIR(1, pxx, Wx, pux)
    LBM_ADJ_PAIR(2, pyy, Wy, puy)
    LBM_ADJ_PAIR(3, pzz, Wz, puz)
    LBM_ADJ_PAIR(4, pxx + pyy + R(2) * pxy, Wx + Wy, pux + puy)
    LBM_ADJ_PAIR(5, pxx + pzz + R(2) * pxz, Wx + Wz, pux + puz)
    LBM_ADJ_PAIR(6, pyy + pzz + R(2) * pyz, Wy + Wz, puy + puz)
    LBM_ADJ_PAIR(7, pxx + pyy - R(2) * pxy, Wx - Wy, pux - puy)
    LBM_ADJ_PAIR(8, pxx + pzz - R(2) * pxz, Wx - Wz, pux - puz)
    LBM_ADJ_PAIR(9, pyy + pzz - R(2) * pyz, Wy - Wz, puy - puz)
#undef LBM_ADJ_PAIR
}

// Probe sources of one cell: lam += src_p . (M c_j - u)/rho for every
// registered probe p at the cell, in probe order; M = I without rotation,
// M c = c - Omega x c with it (the Coriolis part of F/2 in u).  The probe
// table lists (cell, probe) entries sorted by cell; cell0 is the first cell
// of the cell's 64-cell chunk, whose bit in pr.bits is set.
template <typename R>
__device__ inline void add_probe_sources(const AdjProbes& pr, long long cell, long long cell0, const R* h,
                                         const Phys<R>& P, R* ls)
{
    const R* src = (const R*)pr.src;
    int lo = 0, hi = pr.n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)pr.cell[mid] < cell0) lo = mid + 1;
        else hi = mid;
    }
    bool have = false;
    R inv_rho = R(0), ux = R(0), uy = R(0), uz = R(0);
    for (int e = lo; e < pr.n && (long long)pr.cell[e] < cell0 + 64; e++) {
        if ((long long)pr.cell[e] != cell) continue;
        if (!have) {
            R drho;
            moments_pairs<R, 1>(h, P, drho, ux, uy, uz);
            inv_rho = fast_rcp<R>(P.rho0 + drho);
            have = true;
        }
        const int p = pr.id[e];
        R sx = src[3 * p], sy = src[3 * p + 1], sz = src[3 * p + 2];
        const R su = sx * ux + sy * uy + sz * uz;
        if (P.has_rot) {   // src . (M c) = (M^T src) . c, M^T s = s + (W2 x s)/2
            const R* W2 = P.W2;
            const R ax = sx + R(0.5) * (W2[1] * sz - W2[2] * sy);
            const R ay = sy + R(0.5) * (W2[2] * sx - W2[0] * sz);
            const R az = sz + R(0.5) * (W2[0] * sy - W2[1] * sx);
            sx = ax;
            sy = ay;
            sz = az;
        }
        adj_static_for<0, NQ>([&](auto ic) {
            constexpr int j = decltype(ic)::value;
            constexpr V3 c = dirv(j);
            ls[j] += (R(c.x) * sx + R(c.y) * sy + R(c.z) * sz - su) * inv_rho;
        });
    }
}

__device__ inline bool chunk_has_probe(const AdjProbes& pr, long long chunk)
{
    return pr.src && ((pr.bits[chunk >> 5] >> (chunk & 31)) & 1u);
}

// Adjoint of one cell on the general path (every boundary rule).
template <int K>
__device__ inline void adjoint_cell(const typename Codec<K>::store* __restrict__ f_t,
                                    const typename Codec<K>::real* __restrict__ lam_next,
                                    typename Codec<K>::real* __restrict__ lam, const uint64_t* __restrict__ mask,
                                    const Geo& g, const Phys<typename Codec<K>::real>& P, const AdjProbes& pr, int x,
                                    int y, int z)
{
    using C = Codec<K>;
    using R = typename C::real;
    const long long n = cidx(g, x, y, z);
    if (solid_at(mask, g, x, y, z) || inflow_face_of(g, x, y, z) >= 0) {
#pragma unroll
        for (int j = 0; j < NQ; j++) lam[(long long)j * g.N + n] = R(0);
        return;
    }
    R ls[NQ], h[NQ];
    adj_static_for<0, NQ>([&](auto ic) {
        constexpr int k = decltype(ic)::value;
        ls[k] = adj_gather<R, opp(k), false>(lam_next, mask, g, x, y, z);
    });
#pragma unroll
    for (int i = 0; i < NQ; i++) h[i] = C::dec(f_t[(long long)i * g.N + n]);
    collision_transpose<R>(h, ls, P);
    const long long row = (long long)y + (long long)g.ny * z;
    if (chunk_has_probe(pr, (x >> 6) + (long long)g.ncx * row))
        add_probe_sources<R>(pr, n, n - (x & 63), h, P, ls);
#pragma unroll
    for (int j = 0; j < NQ; j++) lam[(long long)j * g.N + n] = ls[j];
}

// Cells of main_box(g, 1): the transposed streaming reduces to
// lam*_k = lam_next(x + c_k, k), or lam_next(x, opp(k)) when x + c_k is
// solid or beyond a WALL face (halfway bounce-back transposed).  One wave is one
// 64-cell chunk of a row; the slot of each direction is one shared lane
// offset plus a wave-uniform base, selected per lane by the solid lane mask.
//
// With an INFLOW x- face and an OUTFLOW x+ face (adj_x_edges) the waves also
// take the four x-face layers of their rows, with per-lane masks instead of
// the general path (whose scattered reads of these columns would fetch
// lines the row's waves fetch as well):
//   x = 0       an inflow cell: lam = 0;
//   x = 1       the populations moving toward x = 0 land in the inflow cell
//               and are dropped, unless that cell is solid (bounce-back);
//   x = nx - 2  a population bounced back toward x+ also fills the outflow
//               copy of its slot in the face cell x = nx - 1, when fluid;
//   x = nx - 1  a population leaving through the outflow face is dropped
//               unless the cell at nx - 2 is solid (then it is its own
//               bounce-back slot), and one moving to nx - 2 also fills the
//               outflow copy of that slot in the face cell of its row.

template <int K>
__device__ inline void adjoint_wave(const typename Codec<K>::store* __restrict__ f_t,
                                    const typename Codec<K>::real* __restrict__ lam_next,
                                    typename Codec<K>::real* __restrict__ lam, const uint64_t* __restrict__ mask,
                                    const Geo& g, const Phys<typename Codec<K>::real>& P,
                                    const StepOff* __restrict__ otab, const AdjProbes& pr, long long wave)
{
    using C = Codec<K>;
    using R = typename C::real;
    const int lane = threadIdx.x & 63;
    const int cx = (int)(wave % g.ncx);
    const long long row = wave / g.ncx;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    const Box B = main_box(g, 1);
    if (y < B.y0 || y > B.y1 || z < B.z0 || z > B.z1) return;
    const int x = cx * 64 + lane;
    const auto& O = class_offsets(otab, row_class(g, y, z));
    // masks from the cached mask rows (the adjoint arrays are 32-bit or wider)
    RowWin W;
    load_rows(W, mask, g, cx, y, z);
    const uint64_t own = W.c[1][1];
    uint64_t any = 0;
    adj_static_for<1, NQ>([&](auto ic) { any |= solid_src_mask<decltype(ic)::value>(W); });
    const bool solid_any = uniform_u64(any) != 0;
    const bool xe = adj_x_edges(g);
    if (x >= g.nx || (!xe && (x < B.x0 || x > B.x1))) return;
    const long long cell = (long long)x + (long long)g.nx * row;
    const uint32_t off = (uint32_t)cell * (uint32_t)sizeof(R);
    const char* lbase = (const char*)lam_next;
    // lane masks of the x-face layers in this chunk (wave-uniform)
    const int base = cx * 64;
    const uint64_t e0 = (xe && base == 0) ? 1ull : 0ull;
    const uint64_t e1 = (xe && base == 0) ? 2ull : 0ull;
    const int lb = g.nx - 2 - base, la = g.nx - 1 - base;
    const uint64_t eb = (xe && lb >= 0 && lb < 64) ? 1ull << lb : 0ull;
    const uint64_t ea = (xe && la >= 0 && la < 64) ? 1ull << la : 0ull;
    // a solid lane (and the inflow cell x = 0) stores 0 with the same store
    // instructions as the rest
    const bool solid_lane = ((own | e0) >> lane) & 1ull;
    R ls[NQ], h[NQ];
    if ((e0 | e1 | eb | ea) != 0) {
        const uint64_t xm_solid = solid_src_mask<1>(W);   // cell x - 1 of the row is solid
        const uint64_t xp_solid = solid_src_mask<2>(W);   // cell x + 1 of the row is solid
        // every slot first, without branches, so that the loads issue together;
        // lanes whose value is their own slot or nothing read the own slot
        uint32_t so[NQ];
        adj_static_for<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            if constexpr (I == 0) {
                so[0] = off;
                ls[0] = *(const R*)(lbase + off);
            } else {
                constexpr V3 c = dirv(I);
                uint64_t force = e0;
                if constexpr (c.x == 1) force |= e1;
                if constexpr (c.x == -1) force |= ea;
                so[I] = lane_select(off + O.on[I], off + O.oo[I], solid_src_mask<I>(W) | force);
                ls[opp(I)] = *(const R*)(lbase + O.lo[I] + so[I]);
            }
        });
        // the outflow copies: the slot at nx - 2 of a population moving to
        // nx - 2 from the face cell, and its copy one cell further in x
        if (ea != 0) {
            R pv[NQ];
            adj_static_for<1, NQ>([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                constexpr V3 c = dirv(I);
                if constexpr (c.x == 1) {
                    const uint64_t part = ea & ~solid_src_mask<I>(W) & ~W.c[1 - c.z][1 - c.y];
                    pv[I] = *(const R*)(lbase + O.lo[I] + lane_select(so[I], so[I] + (uint32_t)sizeof(R), part));
                }
            });
            adj_static_for<1, NQ>([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                constexpr V3 c = dirv(I);
                if constexpr (c.x == 1) {
                    const uint64_t part = ea & ~solid_src_mask<I>(W) & ~W.c[1 - c.z][1 - c.y];
                    if ((part >> lane) & 1ull) ls[opp(I)] += pv[I];
                }
            });
        }
        adj_static_for<1, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            constexpr V3 c = dirv(I);
            const uint64_t sm = solid_src_mask<I>(W);
            if constexpr (c.x == 1) {
                if (((e1 & ~sm) >> lane) & 1ull) ls[opp(I)] = R(0);
            }
            if constexpr (c.x == -1) {
                if (((ea & ~xm_solid) >> lane) & 1ull) ls[opp(I)] = R(0);
                // the own slot of a bounce-back at nx - 2 and its copy (rare:
                // a solid next to the outflow face)
                const uint64_t part = eb & sm & ~xp_solid;
                if (uniform_u64(part) != 0) {
                    const R q = *(const R*)(lbase + O.lo[I] + lane_select(so[I], so[I] + (uint32_t)sizeof(R), part));
                    if ((part >> lane) & 1ull) ls[opp(I)] += q;
                }
            }
        });
    } else if (!solid_any) {
        adj_static_for<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            ls[opp(I)] = *(const R*)(lbase + O.odd[I] + off);
        });
    } else {
        adj_static_for<0, NQ>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            if constexpr (I == 0) {
                ls[0] = *(const R*)(lbase + off);
            } else {
                const uint32_t so = lane_select(off + O.on[I], off + O.oo[I], solid_src_mask<I>(W));
                ls[opp(I)] = *(const R*)(lbase + O.lo[I] + so);
            }
        });
    }
    if (!solid_lane) {
#pragma unroll
        // f(t) is read once and lam(t) written once per step: streaming
        // (non-temporal) hints, 286 -> 266 us per step on the 256x256x96
        // grid (either alone gains half of that)
        for (int i = 0; i < NQ; i++) h[i] = C::dec(__builtin_nontemporal_load(f_t + (long long)i * g.N + cell));
    } else {
#pragma unroll
        for (int i = 0; i < NQ; i++) h[i] = R(0);
    }
    collision_transpose<R>(h, ls, P);
    if (chunk_has_probe(pr, wave) && !solid_lane) add_probe_sources<R>(pr, cell, cell - lane, h, P, ls);
#pragma unroll
    for (int j = 0; j < NQ; j++) __builtin_nontemporal_store(solid_lane ? R(0) : ls[j], lam + (long long)j * g.N + cell);
}

// dL/du_in(face F, height z): the sum over the face's inflow cells at that
// height of lam*_k d feq_k/du at each cell's own inflow velocity (the
// derivative with respect to a shift of the whole row).  One block per
// (F, z): wavefront reductions over the cells and the block's waves in
// order, then a compensated (Neumaier) update of g[0] (sum) and g[1]
// (compensation).
constexpr int ADJ_RED = 256;

template <int K>
__device__ inline void adjoint_inflow(const typename Codec<K>::real* __restrict__ lam_next,
                                      const uint64_t* __restrict__ mask, const double* __restrict__ uin,
                                      const Geo& g, const Phys<typename Codec<K>::real>& P, int F, int zz,
                                      typename Codec<K>::real* gacc)
{
    using R = typename Codec<K>::real;
    const int a = F >> 1;
    // cells of face F at height zz
    long long count;
    if (a == 0) count = g.ny;
    else if (a == 1) count = g.nx;
    else count = ((F & 1) ? g.nz - 1 : 0) == zz ? (long long)g.nx * g.ny : 0;
    R acc[3] = {R(0), R(0), R(0)};
    for (long long t = threadIdx.x; t < count; t += ADJ_RED) {
        int x, y, z = zz;
        if (a == 0) { x = (F & 1) ? g.nx - 1 : 0; y = (int)t; }
        else if (a == 1) { y = (F & 1) ? g.ny - 1 : 0; x = (int)t; }
        else { x = (int)(t % g.nx); y = (int)(t / g.nx); }
        if (solid_at(mask, g, x, y, z) || inflow_face_of(g, x, y, z) != F) continue;
        R ux, uy, uz;   // the cell's own inflow velocity
        load_inflow<R>(uin, g, F, x, y, z, ux, uy, uz);
        adj_static_for<0, NQ>([&](auto ic) {
            constexpr int k = decltype(ic)::value;
            constexpr V3 c = dirv(k);
            const R l = adj_gather<R, opp(k), true>(lam_next, mask, g, x, y, z);
            const R e = R(c.x) * ux + R(c.y) * uy + R(c.z) * uz;
            const R wl = weight<R>(k) * P.rho0 * l;
            acc[0] += wl * (R(3) * R(c.x) + R(9) * e * R(c.x) - R(3) * ux);
            acc[1] += wl * (R(3) * R(c.y) + R(9) * e * R(c.y) - R(3) * uy);
            acc[2] += wl * (R(3) * R(c.z) + R(9) * e * R(c.z) - R(3) * uz);
        });
    }
    constexpr int NW = ADJ_RED / 64;
    __shared__ R sh[3][NW];
    for (int k = 0; k < 3; k++) {
        const R w = wave_sum(acc[k]);
        if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x < 3 && count > 0) {
        const long long o = ((long long)F * g.nz + zz) * 3 + threadIdx.x;
        const long long o2 = 6ll * g.nz * 3 + o;
        R xv = sh[threadIdx.x][0];
        for (int w = 1; w < NW; w++) xv += sh[threadIdx.x][w];
        const R s = gacc[o];
        const R tsum = s + xv;
        R comp = gacc[o2];
        if (fabs((double)s) >= fabs((double)xv)) comp += (s - tsum) + xv;
        else comp += (xv - tsum) + s;
        gacc[o] = tsum;
        gacc[o2] = comp;
    }
}

// One adjoint step in one launch, blocks in the order of the context's
// block schedule: per-cell blocks take the listed face-shell cells on the
// general path, inflow blocks the inflow gradient (one per INFLOW face and
// height; none without g), wave blocks the waves of main_box(g, 1) (whole
// rows of it when adj_x_edges holds).  All of
// them only read f_t and lam_next and write disjoint parts of lam and g, so
// the latency-bound per-cell and inflow blocks run alongside the interior,
// each next to the wave blocks of its rows.
template <int K>
__global__ void __launch_bounds__(256, K == 0 ? 3 : 4)
k_adjoint(const typename Codec<K>::store* __restrict__ f_t, const typename Codec<K>::real* __restrict__ lam_next,
          typename Codec<K>::real* __restrict__ lam, const uint64_t* __restrict__ mask,
          const double* __restrict__ uin, Geo g, Phys<typename Codec<K>::real> P, const StepOff* __restrict__ otab,
          long long nwaves, const unsigned* __restrict__ cells, long long ncells, const unsigned* __restrict__ sched,
          typename Codec<K>::real* gacc, AdjProbes pr)
{
    const unsigned code = sched[blockIdx.x];
    const unsigned b = code & 0x3fffffffu;
    const unsigned kind = code >> 30;
    if (kind == 0) {
        const long long t = b * 256ll + threadIdx.x;
        if (t >= ncells) return;
        const long long n = cells[t];
        const long long row = n / g.nx;
        adjoint_cell<K>(f_t, lam_next, lam, mask, g, P, pr, (int)(n % g.nx), (int)(row % g.ny), (int)(row / g.ny));
        return;
    }
    if (kind == 1) {
        if (!gacc) return;
        const int k = (int)(b / (unsigned)g.nz);
        const int zz = (int)(b % (unsigned)g.nz);
        int F = 0;
#pragma unroll
        for (int q = 0, seen = 0; q < 6; q++)
            if (g.face[q] == F_INFLOW && seen++ == k) F = q;
        adjoint_inflow<K>(lam_next, mask, uin, g, P, F, zz, gacc);
        return;
    }
    const long long wave = (long long)b * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    adjoint_wave<K>(f_t, lam_next, lam, mask, g, P, otab, pr, wave);
}

template <int K>
static hipError_t adjoint_k(const DevCtx& d, const void* f_t, const void* lam_next, void* lam,
                            const void* probe_src, void* g_inflow, hipStream_t s)
{
    using C = Codec<K>;
    using R = typename C::real;
    const Geo& g = d.g;
    const long long nwaves = (long long)g.ncx * g.ny * g.nz;
    AdjProbes pr = d.probes;
    pr.src = pr.n > 0 ? probe_src : nullptr;
    // Four blocks (16 waves) resident per CU: measured fastest for the 32-bit
    // adjoint (with five or more, the waves' gathers of lam(t+1) and loads of
    // f(t) evict each other's lines; with three, latency is exposed).  The
    // registers allow five, so the launch requests enough LDS to leave room
    // for four.  FP64 needs registers for fewer than four anyway.
    size_t lds = 0;
    if (K != 0 && d.lds_per_cu > 0) {
        const size_t stat = 3 * (ADJ_RED / 64) * sizeof(R);   // the inflow blocks' reduction buffer
        const size_t quarter = (size_t)d.lds_per_cu / 4 / 1024 * 1024;
        if (quarter > stat + 1024) lds = quarter - stat;
    }
    hipLaunchKernelGGL((k_adjoint<K>), dim3(d.adj_sched_n), dim3(256), lds, s, (const typename C::store*)f_t,
                       (const R*)lam_next, (R*)lam, d.mask, d.uin, g, phys_of<K>(d), d.off_adj, nwaves, d.adj_list,
                       d.adj_list_n, d.adj_sched, (R*)g_inflow, pr);
    return hipGetLastError();
}

hipError_t launch_adjoint(const DevCtx& d, const void* f_t, const void* lam_next, void* lam, const void* probe_src,
                          void* g_inflow, hipStream_t s)
{
    switch (d.codec) {
        case 0: return adjoint_k<0>(d, f_t, lam_next, lam, probe_src, g_inflow, s);
        case 1: return adjoint_k<1>(d, f_t, lam_next, lam, probe_src, g_inflow, s);
        case 2: return adjoint_k<2>(d, f_t, lam_next, lam, probe_src, g_inflow, s);
        case 3: return adjoint_k<3>(d, f_t, lam_next, lam, probe_src, g_inflow, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
