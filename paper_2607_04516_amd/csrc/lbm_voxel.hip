// Ray-parity voxelizer (Sec. 4.1: axis-aligned rays through the grid
// columns, ray-triangle intersections, odd-even parity along each column,
// independent passes along different ray directions corroborating the
// labels; Sec. 2.1: the solid mask is the Boolean union of the layers).
//
// One thread per ray: rays are cast through the cell centres along the pass
// axis, one per column of the other two axes (u, v); a block is a 64 x 4
// tile of rays, so a wave shares one tile's list of candidate meshes (built
// on the host from the meshes' projected bounding boxes) and reads the
// triangles by broadcast.  Per mesh the thread toggles the cells above each
// crossing in a register bitmask of its ray (parity), then ORs the result
// into the ray's inside mask; the cells set go to a per-pass bit of a byte
// array, and a last kernel takes the majority of the passes.  Everything in
// FP64 with contraction off, in the same order of operations as the stated
// definition, so the labels are exact functions of the input.
#include "lbm.h"
#include "lbm_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#pragma clang fp contract(off)

namespace lbm {

namespace {

constexpr int TILE_U = 64, TILE_V = 4;
constexpr int MAX_RAY = 1024;   // cells along one ray (16 words of bits)

__device__ inline double edge_fn(double pu, double pv, double au, double av, double bu, double bv)
{
    return (bu - au) * (pv - av) - (bv - av) * (pu - au);
}

// A ray foot with edge value e counts for edge A -> B of a counter-clockwise
// triangle when strictly inside, or on an edge that runs upward or
// horizontally toward -u (a shared edge counts for one triangle only).
__device__ inline bool edge_counts(double e, double au, double av, double bu, double bv)
{
    return e > 0.0 || (e == 0.0 && (bv > av || (bv == av && bu < au)));
}

template <int W>
__global__ void __launch_bounds__(TILE_U * TILE_V)
k_vox_pass(const double* __restrict__ tri, const int* __restrict__ starts, const int* __restrict__ tile_off,
           const int* __restrict__ tile_mesh, int ua, int va, int ta, int nu, int nv, int nt, int ntu, long long su,
           long long sv, long long st, uint8_t* __restrict__ out, uint8_t bit)
{
    const int i = blockIdx.x * TILE_U + threadIdx.x;
    const int j = blockIdx.y * TILE_V + threadIdx.y;
    const int tile = blockIdx.y * ntu + blockIdx.x;
    const double pu = i + 0.5, pv = j + 0.5;
    uint64_t inside[W];
#pragma unroll
    for (int w = 0; w < W; w++) inside[w] = 0;
    const int m_end = tile_off[tile + 1];
    for (int q = tile_off[tile]; q < m_end; q++) {
        const int m = tile_mesh[q];
        uint64_t par[W];
#pragma unroll
        for (int w = 0; w < W; w++) par[w] = 0;
        for (int k = starts[m]; k < starts[m + 1]; k++) {
            const double* p = tri + 9 * (long long)k;
            double A[3] = {p[0], p[1], p[2]}, B[3] = {p[3], p[4], p[5]}, C[3] = {p[6], p[7], p[8]};
            const double Au = ua == 0 ? A[0] : (ua == 1 ? A[1] : A[2]);
            const double Av = va == 0 ? A[0] : (va == 1 ? A[1] : A[2]);
            const double At = ta == 0 ? A[0] : (ta == 1 ? A[1] : A[2]);
            double Bu = ua == 0 ? B[0] : (ua == 1 ? B[1] : B[2]);
            double Bv = va == 0 ? B[0] : (va == 1 ? B[1] : B[2]);
            double Bt = ta == 0 ? B[0] : (ta == 1 ? B[1] : B[2]);
            double Cu = ua == 0 ? C[0] : (ua == 1 ? C[1] : C[2]);
            double Cv = va == 0 ? C[0] : (va == 1 ? C[1] : C[2]);
            double Ct = ta == 0 ? C[0] : (ta == 1 ? C[1] : C[2]);
            const double area = edge_fn(Cu, Cv, Au, Av, Bu, Bv);
            if (area == 0.0) continue;   // seen edge-on
            if (area < 0.0) {            // counter-clockwise in the projection
                double tmp;
                tmp = Bu; Bu = Cu; Cu = tmp;
                tmp = Bv; Bv = Cv; Cv = tmp;
                tmp = Bt; Bt = Ct; Ct = tmp;
            }
            const double w0 = edge_fn(pu, pv, Bu, Bv, Cu, Cv);
            const double w1 = edge_fn(pu, pv, Cu, Cv, Au, Av);
            const double w2 = edge_fn(pu, pv, Au, Av, Bu, Bv);
            if (!(edge_counts(w0, Bu, Bv, Cu, Cv) && edge_counts(w1, Cu, Cv, Au, Av) &&
                  edge_counts(w2, Au, Av, Bu, Bv)))
                continue;
            const double t = (w0 * At + w1 * Bt + w2 * Ct) / (w0 + w1 + w2);
            // first cell whose centre lies above the crossing (k + 1/2 > t)
            double fk = floor(t - 0.5) + 1.0;
            fk = fk < 0.0 ? 0.0 : (fk > (double)nt ? (double)nt : fk);
            int k0 = (int)fk;
            while (k0 > 0 && (double)(k0 - 1) + 0.5 > t) k0--;
            while (k0 < nt && !((double)k0 + 0.5 > t)) k0++;
#pragma unroll
            for (int w = 0; w < W; w++) {
                const int lo = 64 * w;
                par[w] ^= k0 <= lo ? ~0ull : (k0 < lo + 64 ? (~0ull << (k0 - lo)) : 0ull);
            }
        }
#pragma unroll
        for (int w = 0; w < W; w++) inside[w] |= par[w];
    }
    if (i >= nu || j >= nv) return;
    const long long base = (long long)i * su + (long long)j * sv;
#pragma unroll
    for (int w = 0; w < W; w++) {
        uint64_t word = inside[w];
        if (64 * (w + 1) > nt) word &= 64 * w >= nt ? 0ull : (~0ull >> (64 * (w + 1) - nt));
        while (word) {
            const int b = __builtin_ctzll(word);
            word &= word - 1;
            out[base + (long long)(64 * w + b) * st] |= bit;
        }
    }
}

__global__ void k_vox_vote(const uint8_t* __restrict__ votes, uint8_t* __restrict__ solid, long long n, int passes)
{
    const long long c = blockIdx.x * 256ll + threadIdx.x;
    if (c >= n) return;
    const uint8_t v = votes[c];
    const bool in = passes == 1 ? (v & 1) != 0 : (((v & 1) + ((v >> 1) & 1) + ((v >> 2) & 1)) >= 2);
    if (in) solid[c] = 1;
}

template <int W>
hipError_t launch_pass(const double* tri, const int* starts, const int* toff, const int* tmesh, int ua, int va, int ta,
                       const int* n, const long long* stride, uint8_t* out, uint8_t bit)
{
    const int nu = n[ua], nv = n[va], nt = n[ta];
    const int ntu = (nu + TILE_U - 1) / TILE_U, ntv = (nv + TILE_V - 1) / TILE_V;
    hipLaunchKernelGGL((k_vox_pass<W>), dim3(ntu, ntv), dim3(TILE_U, TILE_V), 0, 0, tri, starts, toff, tmesh, ua, va,
                       ta, nu, nv, nt, ntu, stride[ua], stride[va], stride[ta], out, bit);
    return hipGetLastError();
}

}  // namespace

// Host part: validation, tile lists, device buffers, passes, vote.
int voxelize(const lbm_grid* grid, const double* tri, int32_t nt, const int32_t* starts, int32_t nm, int32_t passes,
             uint8_t* solid, std::string& err)
{
    if (!grid || !solid || nt < 0 || nm < 0 || (nt > 0 && !tri) || !starts || (passes != 1 && passes != 3)) {
        err = "bad voxelize arguments (NULL pointer, negative count, or passes not 1 or 3)";
        return LBM_EINVAL;
    }
    const int n[3] = {grid->nx, grid->ny, grid->nz};
    for (int a = 0; a < 3; a++)
        if (n[a] < 1 || ((passes == 3 || a == 2) && n[a] > MAX_RAY)) {
            err = "grid extent along a ray axis outside [1, 1024]";
            return LBM_EINVAL;
        }
    if (starts[0] != 0 || starts[nm] != nt) {
        err = "mesh starts must run from 0 to the triangle count";
        return LBM_EINVAL;
    }
    for (int m = 0; m < nm; m++)
        if (starts[m + 1] < starts[m]) {
            err = "mesh starts must not decrease";
            return LBM_EINVAL;
        }
    for (long long k = 0; k < 9ll * nt; k++)
        if (!std::isfinite(tri[k])) {
            err = "non-finite vertex coordinate";
            return LBM_EINVAL;
        }
    const long long N = (long long)n[0] * n[1] * n[2];
    const long long stride[3] = {1, n[0], (long long)n[0] * n[1]};
    // per pass: tile lists of the meshes whose projected bounding box covers a ray of the tile
    const int axes[3][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}};   // (u, v, t) for rays along z, x, y
    std::vector<std::vector<int>> off(passes), mesh(passes);
    for (int p = 0; p < passes; p++) {
        const int ua = axes[p][0], va = axes[p][1];
        const int ntu = (n[ua] + TILE_U - 1) / TILE_U, ntv = (n[va] + TILE_V - 1) / TILE_V;
        std::vector<std::vector<int>> lists((size_t)ntu * ntv);
        for (int m = 0; m < nm; m++) {
            if (starts[m + 1] == starts[m]) continue;
            double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
            for (int k = starts[m]; k < starts[m + 1]; k++)
                for (int v = 0; v < 3; v++) {
                    const double cu = tri[9ll * k + 3 * v + ua], cv = tri[9ll * k + 3 * v + va];
                    lo[0] = std::min(lo[0], cu); hi[0] = std::max(hi[0], cu);
                    lo[1] = std::min(lo[1], cv); hi[1] = std::max(hi[1], cv);
                }
            // rays i with lo <= i + 1/2 <= hi
            const long long i0 = std::max(0ll, (long long)std::ceil(lo[0] - 0.5));
            const long long i1 = std::min((long long)n[ua] - 1, (long long)std::floor(hi[0] - 0.5));
            const long long j0 = std::max(0ll, (long long)std::ceil(lo[1] - 0.5));
            const long long j1 = std::min((long long)n[va] - 1, (long long)std::floor(hi[1] - 0.5));
            if (i0 > i1 || j0 > j1) continue;
            for (long long tv = j0 / TILE_V; tv <= j1 / TILE_V; tv++)
                for (long long tu = i0 / TILE_U; tu <= i1 / TILE_U; tu++) lists[(size_t)(tv * ntu + tu)].push_back(m);
        }
        off[p].assign(lists.size() + 1, 0);
        for (size_t t = 0; t < lists.size(); t++) {
            off[p][t + 1] = off[p][t] + (int)lists[t].size();
            mesh[p].insert(mesh[p].end(), lists[t].begin(), lists[t].end());
        }
    }
    // device buffers
    double* d_tri = nullptr;
    int *d_starts = nullptr, *d_off = nullptr, *d_mesh = nullptr;
    uint8_t *d_votes = nullptr, *d_solid = nullptr;
    size_t moff = 0, mmesh = 0;
    for (int p = 0; p < passes; p++) {
        moff = std::max(moff, off[p].size());
        mmesh = std::max(mmesh, mesh[p].size());
    }
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (e == hipSuccess && r != hipSuccess) e = r;
    };
    chk(hipMalloc((void**)&d_tri, std::max<size_t>(8, 72 * (size_t)nt)));
    chk(hipMalloc((void**)&d_starts, 4 * ((size_t)nm + 1)));
    chk(hipMalloc((void**)&d_off, 4 * moff));
    chk(hipMalloc((void**)&d_mesh, std::max<size_t>(4, 4 * mmesh)));
    chk(hipMalloc((void**)&d_votes, (size_t)N));
    chk(hipMalloc((void**)&d_solid, (size_t)N));
    if (e == hipSuccess && nt) chk(hipMemcpy(d_tri, tri, 72 * (size_t)nt, hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(hipMemcpy(d_starts, starts, 4 * ((size_t)nm + 1), hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(hipMemcpy(d_solid, solid, (size_t)N, hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(hipMemset(d_votes, 0, (size_t)N));
    for (int p = 0; p < passes && e == hipSuccess; p++) {
        chk(hipMemcpy(d_off, off[p].data(), 4 * off[p].size(), hipMemcpyHostToDevice));
        if (!mesh[p].empty()) chk(hipMemcpy(d_mesh, mesh[p].data(), 4 * mesh[p].size(), hipMemcpyHostToDevice));
        if (e != hipSuccess) break;
        const int ta = axes[p][2], words = (n[ta] + 63) / 64;
        const uint8_t bit = (uint8_t)(1 << p);
        if (words <= 2) chk(launch_pass<2>(d_tri, d_starts, d_off, d_mesh, axes[p][0], axes[p][1], ta, n, stride, d_votes, bit));
        else if (words <= 4) chk(launch_pass<4>(d_tri, d_starts, d_off, d_mesh, axes[p][0], axes[p][1], ta, n, stride, d_votes, bit));
        else if (words <= 8) chk(launch_pass<8>(d_tri, d_starts, d_off, d_mesh, axes[p][0], axes[p][1], ta, n, stride, d_votes, bit));
        else chk(launch_pass<16>(d_tri, d_starts, d_off, d_mesh, axes[p][0], axes[p][1], ta, n, stride, d_votes, bit));
        // the tile lists of the next pass overwrite these buffers
        if (e == hipSuccess) chk(hipDeviceSynchronize());
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_vox_vote, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, 0, d_votes, d_solid, N, passes);
        chk(hipGetLastError());
    }
    if (e == hipSuccess) chk(hipMemcpy(solid, d_solid, (size_t)N, hipMemcpyDeviceToHost));
    (void)hipFree(d_tri);
    (void)hipFree(d_starts);
    (void)hipFree(d_off);
    (void)hipFree(d_mesh);
    (void)hipFree(d_votes);
    (void)hipFree(d_solid);
    if (e != hipSuccess) {
        err = std::string("voxelize: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EHIP;
    }
    return LBM_OK;
}

}  // namespace lbm
