// Synthetic von Karman inflow (App. F, turbulence generation): host set-up of
// the active boundary cells and the Fourier mode tables, device evaluation of
// the series into the per-cell inflow velocity array.
//
// One thread per active cell loops over the modes of its face; the cells are
// ordered face by face, so the lanes of a wave read the same mode row (one
// broadcast load).  The phase k.x - omega t is formed in double precision and
// one sincos per mode serves the three components through the precomputed
// A cos(phi) and A sin(phi) of each mode.
#include "lbm_turbulence.h"

#include <cmath>
#include <new>
#include <utility>

namespace lbm {

namespace {

constexpr int VK_ROW = 10;   // kx, ky, kz, omega, then A cos(phi), A sin(phi) for x, y, z
constexpr int VK_MAX_MODES = 4096;
constexpr double VK_PI = 3.14159265358979323846;

struct VkDev {
    const int* slot;      // per-cell inflow entry (inflow_slot) of each active cell
    const int* face;      // its face: selects the mode table
    const double* xg;     // [3][n] global lattice coordinates
    const double* sigma;  // [n] local fluctuation level
    const double* ub;     // [3][n] mean boundary velocity
    const double* modes;  // [6][nm][VK_ROW]
    int n, nm;
};

// q(x_i, t) for every active cell; with qout NULL, U_b + sigma q goes to uin,
// else q goes to qout [3][n].
__global__ void k_vk_eval(VkDev v, double t, double* __restrict__ uin, double* __restrict__ qout)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    const double* M = v.modes + (long long)v.face[i] * v.nm * VK_ROW;
    const double gx = v.xg[i], gy = v.xg[v.n + i], gz = v.xg[2 * v.n + i];
    double qx = 0.0, qy = 0.0, qz = 0.0;
    for (int m = 0; m < v.nm; m++) {
        const double* r = M + (long long)m * VK_ROW;
        const double b = fma(r[0], gx, fma(r[1], gy, fma(r[2], gz, -r[3] * t)));
        double sn, cs;
        sincos(b, &sn, &cs);
        // A cos(b + phi) = A cos(phi) cos b - A sin(phi) sin b
        qx = fma(r[4], cs, fma(-r[5], sn, qx));
        qy = fma(r[6], cs, fma(-r[7], sn, qy));
        qz = fma(r[8], cs, fma(-r[9], sn, qz));
    }
    if (qout) {
        qout[i] = qx;
        qout[v.n + i] = qy;
        qout[2 * v.n + i] = qz;
        return;
    }
    const double s = v.sigma[i];
    double* u = uin + 3 * (long long)v.slot[i];
    u[0] = fma(s, qx, v.ub[i]);
    u[1] = fma(s, qy, v.ub[v.n + i]);
    u[2] = fma(s, qz, v.ub[2 * v.n + i]);
}

// Linear interpolation between two anchors: U_b + sigma ((1 - al) qa + al qb).
__global__ void k_vk_blend(VkDev v, const double* __restrict__ qa, const double* __restrict__ qb, double al,
                           double* __restrict__ uin)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    const double s = v.sigma[i];
    double* u = uin + 3 * (long long)v.slot[i];
    for (int a = 0; a < 3; a++) {
        const long long k = (long long)a * v.n + i;
        const double q = (1.0 - al) * qa[k] + al * qb[k];
        u[a] = fma(s, q, v.ub[k]);
    }
}

const int kNormal[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

double vk_uniform(uint64_t seed, int r, int m, int j)
{
    const uint64_t x = splitmix64(seed + ((uint64_t)(r + 1) << 32) + 6ull * (uint64_t)m + (uint64_t)j);
    return (double)(x >> 11) * 0x1.0p-53;
}

struct HostCell {
    int face, x, y, z;
    double ub[3];
};

bool solid_host(const std::vector<uint64_t>& bits, const Geo& g, int x, int y, int z)
{
    return (bits[((size_t)y + (size_t)g.ny * z) * g.wpr + (x >> 6)] >> (x & 63)) & 1ull;
}

double dot_n(const double* u, int F)
{
    return u[0] * kNormal[F][0] + u[1] * kNormal[F][1] + u[2] * kNormal[F][2];
}

double norm3(const double* u) { return std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); }

}  // namespace

struct VkGen {
    lbm_turbulence p;
    int n = 0, nm = 0;
    double u_ref = 0.0, e_c[3] = {1.0, 0.0, 0.0};
    void* ibuf = nullptr;   // slot, face
    void* dbuf = nullptr;   // xg, sigma, ub, modes, qa, qb
    VkDev dev{};
    double* qa = nullptr;
    double* qb = nullptr;
    int64_t anchor_a = -1, anchor_b = -1;  // times held in qa, qb (interpolation)
    int64_t applied = -1;                  // anchor last written into uin (hold)
};

void vk_destroy(VkGen* v)
{
    if (!v) return;
    if (v->ibuf) (void)hipFree(v->ibuf);
    if (v->dbuf) (void)hipFree(v->dbuf);
    delete v;
}

int vk_create(VkGen** out, const lbm_turbulence& p, const Geo& g, const std::vector<uint64_t>& bits,
              const std::vector<double>& base, std::string& err)
{
    *out = nullptr;
    if (p.n_modes < 1 || p.n_modes > VK_MAX_MODES) {
        err = "n_modes outside [1, 4096]";
        return LBM_EINVAL;
    }
    if (p.stride < 1) {
        err = "stride below 1";
        return LBM_EINVAL;
    }
    bool fin = std::isfinite(p.length_scale) && std::isfinite(p.intensity) && std::isfinite(p.sigma0);
    for (int a = 0; a < 3; a++) fin = fin && std::isfinite(p.gain[a]) && std::isfinite(p.origin[a]);
    if (!fin || !(p.length_scale > 0.0)) {
        err = "length_scale not positive or a parameter not finite";
        return LBM_EINVAL;
    }

    // 1. active cells: INFLOW_EQ faces other than z-, not solid, one face each
    std::vector<HostCell> cand;
    const int vk_faces[5] = {0, 1, 2, 3, 5};
    for (int F : vk_faces) {
        if (g.face[F] != F_INFLOW) continue;
        const int a = F >> 1;
        const int n1 = a == 0 ? g.ny : g.nx, n2 = a == 2 ? g.ny : g.nz;
        const int fixed = (F & 1) ? (a == 0 ? g.nx : a == 1 ? g.ny : g.nz) - 1 : 0;
        for (int j2 = 0; j2 < n2; j2++)
            for (int j1 = 0; j1 < n1; j1++) {
                const int x = a == 0 ? fixed : j1;
                const int y = a == 0 ? j1 : (a == 1 ? fixed : j2);
                const int z = a == 2 ? fixed : j2;
                if (solid_host(bits, g, x, y, z) || inflow_face_of(g, x, y, z) != F) continue;
                HostCell c{F, x, y, z, {0, 0, 0}};
                for (int k = 0; k < 3; k++) c.ub[k] = base[3 * (size_t)inflow_slot(g, F, x, y, z) + k];
                if (p.inflow_only && !(dot_n(c.ub, F) > 0.0)) continue;
                cand.push_back(c);
            }
    }
    // 2. drop faces whose mean velocity has characteristic speed <= 1e-7
    std::vector<HostCell> cells;
    for (int F : vk_faces) {
        double s[3] = {0, 0, 0};
        long long cnt = 0;
        for (const HostCell& c : cand)
            if (c.face == F) {
                for (int k = 0; k < 3; k++) s[k] += c.ub[k];
                cnt++;
            }
        if (!cnt) continue;
        for (int k = 0; k < 3; k++) s[k] /= (double)cnt;
        const double uc = p.char_normal ? std::fabs(dot_n(s, F)) : norm3(s);
        if (!(uc > 1e-7)) continue;
        for (const HostCell& c : cand)
            if (c.face == F) cells.push_back(c);
    }
    VkGen* v = new (std::nothrow) VkGen();
    if (!v) {
        err = "out of host memory";
        return LBM_ENOMEM;
    }
    v->p = p;
    v->n = (int)cells.size();
    v->nm = p.n_modes;
    // 3. global convection speed and direction
    double su[3] = {0, 0, 0}, sn = 0.0;
    for (const HostCell& c : cells) {
        for (int k = 0; k < 3; k++) su[k] += c.ub[k];
        sn += norm3(c.ub);
    }
    v->u_ref = v->n ? sn / v->n : 0.0;
    const double ns = norm3(su);
    if (ns > 0.0)
        for (int k = 0; k < 3; k++) v->e_c[k] = su[k] / ns;
    if (v->n == 0) {
        *out = v;
        return LBM_OK;
    }

    // 4. mode tables, one per face (or one shared realization)
    const int nm = v->nm;
    std::vector<double> modes((size_t)6 * nm * VK_ROW, 0.0);
    double kmin = 2.0 * VK_PI / (10.0 * p.length_scale);
    const double kmax = VK_PI;
    if (!(kmin < kmax)) kmin = 0.1 * kmax;
    const double lmin = std::log(kmin), lmax = std::log(kmax);
    bool used[6] = {false, false, false, false, false, false};
    for (const HostCell& c : cells) used[c.face] = true;
    for (int F = 0; F < 6; F++) {
        if (!used[F]) continue;
        const int r = p.shared ? 0 : F;
        double* tab = modes.data() + (size_t)F * nm * VK_ROW;
        std::vector<double> amp(nm);
        double sum2 = 0.0;
        for (int m = 0; m < nm; m++) {
            double u[6];
            for (int j = 0; j < 6; j++) u[j] = vk_uniform(p.seed, r, m, j);
            const double xi = ((double)m + u[0]) / nm;
            const double k = std::exp(lmin + xi * (lmax - lmin));
            const double mu = 2.0 * u[1] - 1.0, th = 2.0 * VK_PI * u[2];
            const double st = std::sqrt(1.0 - mu * mu);
            double* row = tab + (size_t)m * VK_ROW;
            row[0] = k * st * std::cos(th);
            row[1] = k * st * std::sin(th);
            row[2] = k * mu;
            row[3] = v->u_ref * (row[0] * v->e_c[0] + row[1] * v->e_c[1] + row[2] * v->e_c[2]);
            const double kl = k * p.length_scale;
            amp[m] = std::sqrt(k * k * k * k / std::pow(1.0 + kl * kl, 17.0 / 6.0));
            sum2 += amp[m] * amp[m];
            for (int a = 0; a < 3; a++) {
                const double ph = 2.0 * VK_PI * u[3 + a];
                row[4 + 2 * a] = std::cos(ph);
                row[5 + 2 * a] = std::sin(ph);
            }
        }
        const double inv = 1.0 / std::sqrt(0.5 * sum2);
        for (int m = 0; m < nm; m++) {
            double* row = tab + (size_t)m * VK_ROW;
            for (int a = 0; a < 3; a++) {
                const double A = amp[m] * inv * p.gain[a];
                row[4 + 2 * a] *= A;
                row[5 + 2 * a] *= A;
            }
        }
    }

    // 5. per-cell data
    const int n = v->n;
    std::vector<int> ih(2 * (size_t)n);
    std::vector<double> dh((size_t)7 * n + modes.size());
    for (int i = 0; i < n; i++) {
        const HostCell& c = cells[i];
        ih[i] = (int)inflow_slot(g, c.face, c.x, c.y, c.z);
        ih[n + i] = c.face;
        dh[i] = p.origin[0] + c.x;
        dh[n + i] = p.origin[1] + c.y;
        dh[2 * (size_t)n + i] = p.origin[2] + c.z;
        const double uc = p.char_normal ? std::fabs(dot_n(c.ub, c.face)) : norm3(c.ub);
        dh[3 * (size_t)n + i] = p.intensity > 0.0 ? p.intensity * uc : p.sigma0;
        for (int k = 0; k < 3; k++) dh[(4 + (size_t)k) * n + i] = c.ub[k];
    }
    std::copy(modes.begin(), modes.end(), dh.begin() + (size_t)7 * n);
    const size_t dbytes = (dh.size() + 6 * (size_t)n) * sizeof(double);
    hipError_t e = hipMalloc(&v->ibuf, ih.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&v->dbuf, dbytes);
    if (e == hipSuccess) e = hipMemcpy(v->ibuf, ih.data(), ih.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(v->dbuf, dh.data(), dh.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        const bool oom = e == hipErrorOutOfMemory;
        (void)hipGetLastError();
        err = std::string("turbulence tables: ") + hipGetErrorString(e);
        vk_destroy(v);
        return oom ? LBM_ENOMEM : LBM_EHIP;
    }
    const int* ib = (const int*)v->ibuf;
    double* db = (double*)v->dbuf;
    v->dev.slot = ib;
    v->dev.face = ib + n;
    v->dev.xg = db;
    v->dev.sigma = db + 3 * (size_t)n;
    v->dev.ub = db + 4 * (size_t)n;
    v->dev.modes = db + 7 * (size_t)n;
    v->dev.n = n;
    v->dev.nm = nm;
    v->qa = db + dh.size();
    v->qb = v->qa + 3 * (size_t)n;
    *out = v;
    return LBM_OK;
}

void vk_invalidate(VkGen* v)
{
    if (!v) return;
    v->anchor_a = v->anchor_b = v->applied = -1;
}

void vk_info(const VkGen* v, int64_t* n_active, double* u_ref, double* e_c)
{
    if (n_active) *n_active = v ? v->n : 0;
    if (u_ref) *u_ref = v ? v->u_ref : 0.0;
    if (e_c)
        for (int k = 0; k < 3; k++) e_c[k] = v ? v->e_c[k] : 0.0;
}

hipError_t vk_apply(VkGen* v, double* uin, int64_t t, hipStream_t s)
{
    if (!v || v->n == 0) return hipSuccess;
    const int64_t st = v->p.stride;
    const unsigned nb = (unsigned)((v->n + 255) / 256);
    if (st <= 1 || !v->p.interpolate) {
        const int64_t ta = st <= 1 ? t : (t / st) * st;
        if (st > 1 && ta == v->applied) return hipSuccess;
        hipLaunchKernelGGL(k_vk_eval, dim3(nb), dim3(256), 0, s, v->dev, (double)ta, uin, (double*)nullptr);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) v->applied = ta;
        return e;
    }
    const int64_t ta = (t / st) * st, tb = ta + st;
    if (v->anchor_a != ta) {
        if (v->anchor_b == ta) {
            std::swap(v->qa, v->qb);
            v->anchor_a = ta;
            v->anchor_b = -1;
        } else {
            hipLaunchKernelGGL(k_vk_eval, dim3(nb), dim3(256), 0, s, v->dev, (double)ta, (double*)nullptr, v->qa);
            v->anchor_a = ta;
        }
    }
    if (v->anchor_b != tb) {
        hipLaunchKernelGGL(k_vk_eval, dim3(nb), dim3(256), 0, s, v->dev, (double)tb, (double*)nullptr, v->qb);
        v->anchor_b = tb;
    }
    const double al = (double)(t - ta) / (double)st;
    hipLaunchKernelGGL(k_vk_blend, dim3(nb), dim3(256), 0, s, v->dev, v->qa, v->qb, al, uin);
    return hipGetLastError();
}

}  // namespace lbm
