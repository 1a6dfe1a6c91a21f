// C-ABI runtime of the D3Q19 LBM-LES library: context lifetime, argument
// validation, device allocation, parity bookkeeping of the in-place A-A
// update, error reporting.  Declarations and contracts are in include/lbm.h.
#include "lbm.h"
#include "lbm_launch.h"
#include "lbm_turbulence.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace lbm;

// Device scratch of lbm_probe_noalloc: the staged probe points [np][3]
// followed by their results [np][4] (floats), one copy per GPU, held until
// the process ends.  Host code never uses the array's name as an address:
// lbm_create looks up each device's copy with hipGetSymbolAddress (device
// current) and keeps the pointer per device.
static __device__ __align__(256) float scratch[LBM_PROBE_NOALLOC_MAX * 7];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};
}  // namespace

struct lbm_ctx {
    DevCtx d;
    lbm_params p;
    hipStream_t stream = nullptr;
    int device = 0;
    int phase = 0;          // 0: natural layout (pre-collision f(t)); 1: swapped (after an even step)
    int64_t t = 0;
    size_t store_bytes = 0; // bytes of one stored population
    void* f = nullptr;
    uint64_t* mask = nullptr;
    void* ghost = nullptr;
    double* ubase = nullptr;  // device per-cell boundary states of the INFLOW_EQ faces [n_in][3] (inflow_slot)
    std::vector<double> base_host;  // host copy of ubase
    double* uin = nullptr;  // device per-cell inflow velocities [n_in][3]: ubase plus turbulence / flux shift
    long long n_in = 0;
    std::vector<uint64_t> bits_host;  // solid bits, kept for the turbulence generator
    VkGen* vk = nullptr;              // synthetic inflow generator, NULL when off
    lbm_turbulence vkp{};
    // flux balancing: boundary cells (inflow entry, face), partial sums, phi
    int flux_mode = 0;
    int* flux_cells = nullptr;        // [2][n_flux]: slot, then face
    long long n_flux = -1;            // -1: list not built yet
    double* flux_red = nullptr;       // partial sums, then phi at the end
    bool prof_set[6] = {false, false, false, false, false, false};
    bool halo[6] = {false, false, false, false, false, false};  // LBM_HALO faces (ghost rows)
    double* u0 = nullptr;   // device [nz][3] scratch for initialisation
    int* probes = nullptr;  // device [np][3]
    int np = 0;
    void* probe_tab = nullptr;  // device: probe table (chunk bits, sorted cells, probe ids)
    bool probe_fold = false;    // every probe is sampled by the fast step kernels (see lbm_set_probes)
    double* red_partial = nullptr;
    double* red_out = nullptr;  // device [5]
    unsigned* odd_list = nullptr;
    unsigned* push_list = nullptr;
    unsigned* adj_list = nullptr;
    unsigned* push_sched = nullptr;  // block order of the push launch
    unsigned* adj_sched = nullptr;   // block order of the adjoint launch
    StepOff* offsets = nullptr;     // [54] row-class slot offsets: odd (x 4 block edges), push, adjoint
    int* wave_idx = nullptr;        // per wave: entry in wave_tab or -1
    uint64_t* wave_tab = nullptr;   // solid-source masks of waves with a solid neighbour
    void* stats = nullptr;
    int stats_stride = 0;
    int64_t fluid = 0, interior = 0;
    // step-kernel timing (lbm_profile): event pairs around each launch
    bool profiling = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    std::string err;
};

static thread_local std::string g_create_error;

static int fail(lbm_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

static int hip_fail(lbm_ctx* c, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, LBM_EHIP, m);
}

#define HIPCHK(ctx, expr, what)                          \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
    } while (0)

static size_t codec_bytes(int s)
{
    switch (s) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        case LBM_F16S:
        case LBM_BF16S: return 2;
        default: return 0;
    }
}

static long long face_cells_host(const Geo& g, int F)
{
    const int a = F >> 1;
    return a == 0 ? (long long)g.ny * g.nz : (a == 1 ? (long long)g.nx * g.nz : (long long)g.nx * g.ny);
}

// Block order of a launch that mixes per-cell blocks (cells of a list, 256
// per block) and inflow-gradient blocks (one per INFLOW face and height)
// with wave blocks (4 chunks of 64 cells each): every block is placed at the
// first row it touches, the per-cell and inflow blocks ahead of the wave
// blocks of that row.  Blocks are dispatched in order, so the scattered
// loads of a per-cell block find the lines the wave blocks of its rows
// fetch at about the same time.  Entry: kind << 30 | index, kind 0 per-cell,
// 1 inflow, 2 wave block.
static std::vector<unsigned> block_schedule(const Geo& g, const std::vector<unsigned>& cells, bool inflow)
{
    struct B {
        long long row;
        unsigned code;
    };
    std::vector<B> b;
    const long long nwaves = (long long)g.ncx * g.ny * g.nz;
    for (size_t s = 0; s * 256 < cells.size(); s++) b.push_back({(long long)(cells[s * 256] / (unsigned)g.nx), (unsigned)s});
    if (inflow) {
        int k = 0;
        for (int F = 0; F < 6; F++) {
            if (g.face[F] != F_INFLOW) continue;
            for (int z = 0; z < g.nz; z++) {
                const int zr = (F >> 1) == 2 ? ((F & 1) ? g.nz - 1 : 0) : z;
                const long long row = (F >> 1) == 1 ? ((F & 1) ? g.ny - 1 : 0) + (long long)g.ny * zr : (long long)g.ny * zr;
                b.push_back({row, (1u << 30) | (unsigned)(k * g.nz + z)});
            }
            k++;
        }
    }
    for (long long m = 0; 4 * m < nwaves; m++) b.push_back({(4 * m) / g.ncx, (2u << 30) | (unsigned)m});
    std::stable_sort(b.begin(), b.end(), [](const B& p, const B& q) {
        return p.row != q.row ? p.row < q.row : (p.code >> 30) < (q.code >> 30);
    });
    std::vector<unsigned> out(b.size());
    for (size_t i = 0; i < b.size(); i++) out[i] = b[i].code;
    return out;
}

// Hardware block i of a launch runs on XCD i % 8, each XCD with its own L2.
// group_on_xcds reorders a block schedule so that G consecutive entries run
// on one XCD: it pads the schedule with no-op entries (a wave block beyond
// the grid, which the kernels skip) to a multiple of 8 G and gives hardware
// block i the entry at (slot / G) 8 G + (i % 8) G + slot % G, slot = i / 8.
// Neighbouring wave blocks of the push and adjoint launches share the lines
// at their chunk and row edges; with G = 4 on the 256x256x96 grid the push
// step took 201 instead of 215 us and the adjoint step 260 instead of 264 us
// (G = 2: 206 / 264, G = 8: 200 / 261, G = 16: 198 / 264).
constexpr int SCHED_XCD_GROUP = 4;

static void group_on_xcds(std::vector<unsigned>& s, long long nwaves, int G)
{
    const unsigned beyond = (unsigned)((nwaves + 3) / 4);
    if (G <= 1 || beyond >= (1u << 30)) return;
    const unsigned noop = (2u << 30) | beyond;
    const size_t m = (size_t)8 * G;
    std::vector<unsigned> p = s;
    while (p.size() % m) p.push_back(noop);
    s.resize(p.size());
    for (size_t i = 0; i < p.size(); i++) {
        const size_t slot = i >> 3, x = i & 7;
        s[i] = p[(slot / G) * m + x * G + slot % G];
    }
}

static bool has_halo(const lbm_ctx* c)
{
    return c->halo[2] || c->halo[3];
}

static void free_all(lbm_ctx* c)
{
    if (!c) return;
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    c->ev_used = 0;
    vk_destroy(c->vk);
    c->vk = nullptr;
    void* ptrs[] = {c->f, c->mask, c->ghost, c->ubase, c->u0, c->probes, c->red_partial, c->red_out, c->odd_list,
                    c->push_list, c->adj_list, c->push_sched, c->adj_sched, c->uin, c->flux_cells, c->flux_red, c->wave_idx, c->wave_tab, c->offsets,
                    c->probe_tab};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    c->f = nullptr;
    c->mask = nullptr;
    c->ghost = nullptr;
    c->ubase = nullptr;
    c->u0 = nullptr;
    c->probes = nullptr;
    c->probe_tab = nullptr;
    c->d.probes = AdjProbes{nullptr, nullptr, nullptr, 0, nullptr};
    c->red_partial = nullptr;
    c->red_out = nullptr;
    c->odd_list = nullptr;
    c->push_list = nullptr;
    c->adj_list = nullptr;
    c->push_sched = nullptr;
    c->adj_sched = nullptr;
    c->uin = nullptr;
    c->flux_cells = nullptr;
    c->flux_red = nullptr;
    c->n_flux = -1;
    c->wave_idx = nullptr;
    c->wave_tab = nullptr;
    c->offsets = nullptr;
}


static int device_alloc(lbm_ctx* c, void** ptr, size_t bytes, const char* what)
{
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 8);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return fail(c, LBM_ENOMEM, std::string("out of device memory allocating ") + what);
    }
    if (e != hipSuccess) return hip_fail(c, e, what);
    return LBM_OK;
}

// Per-wave solid-source masks (static geometry): flags on the device, a
// prefix numbering on the host, then the compact table.
static int build_wave_masks(lbm_ctx* c)
{
    const Geo& g = c->d.g;
    const long long nwaves = (long long)g.ncx * g.ny * g.nz;
    int rc;
    if ((rc = device_alloc(c, (void**)&c->wave_idx, (size_t)nwaves * sizeof(int), "wave masks")) != LBM_OK) return rc;
    HIPCHK(c, launch_wave_masks(c->d, c->wave_idx, nullptr, 0, c->stream), "wave mask flags");
    std::vector<int> h((size_t)nwaves);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->wave_idx, h.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream),
           "wave mask flags");
    HIPCHK(c, hipStreamSynchronize(c->stream), "wave mask flags");
    long long n = 0;
    for (long long w = 0; w < nwaves; w++) h[(size_t)w] = h[(size_t)w] ? (int)n++ : -1;
    if ((rc = device_alloc(c, (void**)&c->wave_tab, (size_t)n * 18 * sizeof(uint64_t), "wave masks")) != LBM_OK)
        return rc;
    HIPCHK(c, hipMemcpyAsync(c->wave_idx, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice, c->stream),
           "wave mask index");
    HIPCHK(c, launch_wave_masks(c->d, c->wave_idx, c->wave_tab, 1, c->stream), "wave mask table");
    HIPCHK(c, hipStreamSynchronize(c->stream), "wave mask table");
    c->d.wave_idx = c->wave_idx;
    c->d.wave_tab = c->wave_tab;
    // slot offsets of the nine row classes: the odd step (in-place row-block
    // layout, per block edge), the push recompute and the adjoint (canonical
    // layout)
    std::vector<StepOff> off(54);
    const int es = (int)c->store_bytes, er = c->p.storage == LBM_F64 ? 8 : 4;
    for (int k = 0; k < 9; k++) {
        for (int e = 0; e < 4; e++) off[4 * k + e] = step_offsets_blocked(g.pitch, g.nyp, g.lrb, es, k, e);
        off[36 + k] = step_offsets(g.N, g.nx, g.ny, es, k);
        off[45 + k] = step_offsets(g.N, g.nx, g.ny, er, k);
    }
    if ((rc = device_alloc(c, (void**)&c->offsets, off.size() * sizeof(StepOff), "slot offsets")) != LBM_OK)
        return rc;
    HIPCHK(c, hipMemcpy(c->offsets, off.data(), off.size() * sizeof(StepOff), hipMemcpyHostToDevice), "slot offsets");
    c->d.off_odd = c->offsets;
    c->d.off_push = c->offsets + 36;
    c->d.off_adj = c->offsets + 45;
    return LBM_OK;
}

static int upload_u0(lbm_ctx* c, const double* u0)
{
    const int nz = c->d.g.nz;
    std::vector<double> h(3 * (size_t)nz);
    for (int z = 0; z < nz; z++)
        for (int a = 0; a < 3; a++) h[3 * z + a] = u0 ? u0[3 * z + a] : c->p.u_init[a];
    HIPCHK(c, hipMemcpyAsync(c->u0, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream), "upload u0");
    HIPCHK(c, hipStreamSynchronize(c->stream), "upload u0");
    return LBM_OK;
}

extern "C" {

int lbm_create(const lbm_grid* grid, const uint8_t* solid, const lbm_params* params, lbm_ctx** out)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!grid || !solid || !params) return fail(nullptr, LBM_EINVAL, "NULL argument");
    if (grid->nx < 3 || grid->ny < 3 || grid->nz < 3) return fail(nullptr, LBM_EINVAL, "each dimension must be >= 3");
    if (!(params->tau0 > 0.5) || !std::isfinite(params->tau0)) return fail(nullptr, LBM_EINVAL, "tau0 must be > 1/2");
    if (!(params->c_smag >= 0.0) || !(params->delta > 0.0) || !(params->rho0 > 0.0))
        return fail(nullptr, LBM_EINVAL, "c_smag must be >= 0, delta and rho0 > 0");
    if (codec_bytes(params->storage) == 0) return fail(nullptr, LBM_EINVAL, "unknown storage codec");
    for (int a = 0; a < 3; a++) {
        const int lo = params->face[2 * a], hi = params->face[2 * a + 1];
        const int top = a == 1 ? LBM_HALO : 4;   // ghost rows: y faces only
        if (lo < 0 || lo > top || hi < 0 || hi > top) return fail(nullptr, LBM_EINVAL, "unknown face kind");
        if ((lo == LBM_PERIODIC) != (hi == LBM_PERIODIC)) return fail(nullptr, LBM_EINVAL, "periodic faces must be paired");
    }
    const long long N = (long long)grid->nx * grid->ny * grid->nz;
    {
        // the step kernels address the two candidate slots of a direction in
        // the in-place array with 32-bit byte offsets from the nearer one: a
        // neighbour in z lies one plane of all 19 populations away
        // (19 pitch nyp elements), plus the block-edge and slot terms
        const long long pitch = ((long long)grid->nx + 63) / 64 * 64;
        int lrb, nyp;
        row_blocks(grid->ny, lrb, nyp);
        const long long span =
            (NQ * pitch * nyp + 40 * 32 * pitch + 2 * pitch) * (long long)codec_bytes(params->storage);
        if (span >= (1ll << 32) || (long long)grid->ny * grid->nz * (((long long)grid->nx + 63) / 64) >= (1ll << 32))
            return fail(nullptr, LBM_EINVAL,
                        "grid too large for one context (19 populations of one xy plane must stay below 4 GiB)");
    }

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
    c->p = *params;
    c->stream = (hipStream_t)params->hip_stream;
    c->store_bytes = codec_bytes(params->storage);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, LBM_EHIP, "no HIP device");
    }
    if (c->device < 0 || c->device >= kMaxDevices) {
        delete c;
        return fail(nullptr, LBM_EINVAL, "device ordinal beyond the library's limit");
    }
    {
        // this device's copy of the lbm_probe_noalloc scratch (once per device)
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch[c->device]) {
            void* ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) {
                delete c;
                return fail(nullptr, LBM_EHIP, std::string("scratch lookup: ") + hipGetErrorString(e));
            }
            g_scratch[c->device] = (float*)ptr;
        }
    }
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device) != hipSuccess)
            lds = 0;
        c->d.lds_per_cu = lds;
    }

    Geo& g = c->d.g;
    g.nx = grid->nx;
    g.ny = grid->ny;
    g.nz = grid->nz;
    g.ncx = (g.nx + 63) / 64;
    g.pitch = g.ncx * 64;
    g.wpr = g.ncx;
    // rows per block of the in-place array (each xy plane padded to whole blocks)
    row_blocks(g.ny, g.lrb, g.nyp);
    // a ghost row is updated like a free-slip face row (its values are
    // replaced or discarded by the halo exchange)
    for (int k = 0; k < 6; k++) {
        c->halo[k] = params->face[k] == LBM_HALO;
        g.face[k] = c->halo[k] ? F_FREESLIP : params->face[k];
    }
    g.S = (long long)g.pitch * g.nyp * g.nz;
    g.N = N;
    long long goff = 0;
    for (int F = 0; F < 6; F++) {
        g.ghost_off[F] = goff;
        if (g.face[F] == LBM_OUTFLOW_ZG) goff += 5 * face_cells_host(g, F);
    }
    for (int F = 0; F < 6; F++) {
        g.in_off[F] = -1;
        if (g.face[F] == LBM_INFLOW_EQ) {
            g.in_off[F] = c->n_in;
            c->n_in += face_cells_host(g, F);
        }
    }
    c->d.codec = params->storage;
    c->d.tau0 = params->tau0;
    c->d.c_smag = params->c_smag;
    c->d.delta = params->delta;
    c->d.rho0 = params->rho0;
    for (int a = 0; a < 3; a++) {
        c->d.force[a] = params->body_force[a];
        c->d.omega[a] = 0.0;
    }
    c->d.sponge_w = 0;
    c->d.sponge_s = 0.0;

    // bit-packed solid mask, cell counts
    std::vector<uint64_t> bits((size_t)g.wpr * g.ny * g.nz, 0ull);
    auto is_inflow = [&](int x, int y, int z) {
        return (g.face[0] == LBM_INFLOW_EQ && x == 0) || (g.face[1] == LBM_INFLOW_EQ && x == g.nx - 1) ||
               (g.face[2] == LBM_INFLOW_EQ && y == 0) || (g.face[3] == LBM_INFLOW_EQ && y == g.ny - 1) ||
               (g.face[4] == LBM_INFLOW_EQ && z == 0) || (g.face[5] == LBM_INFLOW_EQ && z == g.nz - 1);
    };
    for (int z = 0; z < g.nz; z++)
        for (int y = 0; y < g.ny; y++)
            for (int x = 0; x < g.nx; x++) {
                const size_t n = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * z);
                if (solid[n]) {
                    bits[((size_t)y + (size_t)g.ny * z) * g.wpr + (x >> 6)] |= 1ull << (x & 63);
                } else {
                    c->fluid++;
                    if (!is_inflow(x, y, z)) c->interior++;
                }
            }

    int rc;
    const size_t pop_bytes = (size_t)NQ * (size_t)g.S * c->store_bytes;
    if ((rc = device_alloc(c, &c->f, pop_bytes, "populations")) != LBM_OK ||
        (rc = device_alloc(c, (void**)&c->mask, bits.size() * sizeof(uint64_t), "mask")) != LBM_OK ||
        (rc = device_alloc(c, &c->ghost, (size_t)goff * c->store_bytes, "ghost planes")) != LBM_OK ||
        (rc = device_alloc(c, (void**)&c->ubase, 3 * (size_t)c->n_in * sizeof(double), "boundary states")) != LBM_OK ||
        (rc = device_alloc(c, (void**)&c->u0, 3 * (size_t)g.nz * sizeof(double), "u0")) != LBM_OK ||
        (rc = device_alloc(c, (void**)&c->uin, 3 * (size_t)c->n_in * sizeof(double), "inflow velocities")) != LBM_OK ||
        (rc = device_alloc(c, (void**)&c->red_partial, 5 * (size_t)mass_blocks(g) * sizeof(double), "reduction")) !=
            LBM_OK ||
        (rc = device_alloc(c, (void**)&c->red_out, 8 * sizeof(double), "reduction")) != LBM_OK) {
        g_create_error = c->err;
        free_all(c);
        delete c;
        return rc;
    }
    // waves of the odd step handled by the general kernel
    std::vector<unsigned> olist;
    for (int z = 0; z < g.nz; z++)
        for (int y = 0; y < g.ny; y++)
            for (int cx = 0; cx < g.ncx; cx++)
                if (odd_wave_is_general(g, cx, y, z))
                    olist.push_back((unsigned)(cx + (long long)g.ncx * (y + (long long)g.ny * z)));
    if ((rc = device_alloc(c, (void**)&c->odd_list, olist.size() * sizeof(unsigned), "wave list")) != LBM_OK) {
        g_create_error = c->err;
        free_all(c);
        delete c;
        return rc;
    }
    if (!olist.empty() &&
        hipMemcpy(c->odd_list, olist.data(), olist.size() * sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess) {
        g_create_error = "upload wave list";
        free_all(c);
        delete c;
        return LBM_EHIP;
    }
    c->d.odd_list = c->odd_list;
    c->d.odd_list_n = (long long)olist.size();
    // cells outside the fast kernels' boxes (main_box): general path
    std::vector<unsigned> plist, alist;
    for (int z = 0; z < g.nz; z++)
        for (int y = 0; y < g.ny; y++)
            for (int x = 0; x < g.nx; x++) {
                const unsigned n = (unsigned)(x + (long long)g.nx * (y + (long long)g.ny * z));
                const Box bp = main_box(g, 0), ba = main_box(g, 1);
                // the push's waves take the x-face cells of some rows as well
                const bool pin = (x >= bp.x0 && x <= bp.x1) || push_x_edge_row(g, params->storage <= LBM_F32, y, z);
                if (!pin || y < bp.y0 || y > bp.y1 || z < bp.z0 || z > bp.z1) plist.push_back(n);
                // with an inflow x- face and an outflow x+ face the adjoint's
                // waves take their rows' x-face layers as well
                const bool xin = adj_x_edges(g) || (x >= ba.x0 && x <= ba.x1);
                if (!xin || y < ba.y0 || y > ba.y1 || z < ba.z0 || z > ba.z1) alist.push_back(n);
            }
    if ((rc = device_alloc(c, (void**)&c->push_list, plist.size() * sizeof(unsigned), "cell list")) != LBM_OK ||
        (rc = device_alloc(c, (void**)&c->adj_list, alist.size() * sizeof(unsigned), "cell list")) != LBM_OK) {
        g_create_error = c->err;
        free_all(c);
        delete c;
        return rc;
    }
    if (hipMemcpy(c->push_list, plist.data(), plist.size() * sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->adj_list, alist.data(), alist.size() * sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess) {
        g_create_error = "upload cell lists";
        free_all(c);
        delete c;
        return LBM_EHIP;
    }
    c->d.push_list = c->push_list;
    c->d.push_list_n = (long long)plist.size();
    c->d.adj_list = c->adj_list;
    c->d.adj_list_n = (long long)alist.size();
    {
        std::vector<unsigned> sp = block_schedule(g, plist, false), sa = block_schedule(g, alist, true);
        group_on_xcds(sp, (long long)g.ncx * g.ny * g.nz, SCHED_XCD_GROUP);
        group_on_xcds(sa, (long long)g.ncx * g.ny * g.nz, SCHED_XCD_GROUP);
        if ((rc = device_alloc(c, (void**)&c->push_sched, sp.size() * sizeof(unsigned), "block order")) != LBM_OK ||
            (rc = device_alloc(c, (void**)&c->adj_sched, sa.size() * sizeof(unsigned), "block order")) != LBM_OK) {
            g_create_error = c->err;
            free_all(c);
            delete c;
            return rc;
        }
        if (hipMemcpy(c->push_sched, sp.data(), sp.size() * sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->adj_sched, sa.data(), sa.size() * sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess) {
            g_create_error = "upload block order";
            free_all(c);
            delete c;
            return LBM_EHIP;
        }
        c->d.push_sched = c->push_sched;
        c->d.push_sched_n = (unsigned)sp.size();
        c->d.adj_sched = c->adj_sched;
        c->d.adj_sched_n = (unsigned)sa.size();
    }
    c->base_host.assign(3 * (size_t)c->n_in, 0.0);
    hipError_t e = hipMemcpy(c->mask, bits.data(), bits.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && c->n_in) e = hipMemset(c->ubase, 0, 3 * (size_t)c->n_in * sizeof(double));
    if (e == hipSuccess && c->n_in) e = hipMemset(c->uin, 0, 3 * (size_t)c->n_in * sizeof(double));
    if (e == hipSuccess) e = hipMemset(c->f, 0, pop_bytes);
    if (e == hipSuccess && goff) e = hipMemset(c->ghost, 0, (size_t)goff * c->store_bytes);
    if (e != hipSuccess) {
        hip_fail(nullptr, e, "upload");
        free_all(c);
        delete c;
        return LBM_EHIP;
    }
    c->d.f = c->f;
    c->d.mask = c->mask;
    c->d.ghost = c->ghost;
    c->d.ubase = c->ubase;
    c->d.uin = c->uin;
    c->bits_host = std::move(bits);
    if ((rc = build_wave_masks(c)) != LBM_OK) {
        g_create_error = c->err;
        free_all(c);
        delete c;
        return rc;
    }
    if ((rc = lbm_reset(c, nullptr)) != LBM_OK) {
        g_create_error = c->err;
        free_all(c);
        delete c;
        return rc;
    }
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

const char* lbm_last_error(const lbm_ctx* c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

int lbm_cell_counts(const lbm_ctx* c, int64_t* fluid, int64_t* interior)
{
    if (!c) return LBM_EINVAL;
    if (fluid) *fluid = c->fluid;
    if (interior) *interior = c->interior;
    return LBM_OK;
}

int lbm_layout(const lbm_ctx* c, int32_t* rows_per_block, int32_t* ny_pad, int32_t* nx_pitch)
{
    if (!c) return LBM_EINVAL;
    if (rows_per_block) *rows_per_block = 1 << c->d.g.lrb;
    if (ny_pad) *ny_pad = c->d.g.nyp;
    if (nx_pitch) *nx_pitch = c->d.g.pitch;
    return LBM_OK;
}

int lbm_set_stream(lbm_ctx* c, void* s)
{
    if (!c) return LBM_EINVAL;
    c->stream = (hipStream_t)s;
    c->p.hip_stream = s;
    return LBM_OK;
}

// Copy the boundary states of face F (host) into ubase and uin (device).
static int upload_base(lbm_ctx* c, int F)
{
    const Geo& g = c->d.g;
    if (g.in_off[F] < 0) return LBM_OK;
    const size_t off = 3 * (size_t)g.in_off[F], n = 3 * (size_t)face_cells_host(g, F);
    HIPCHK(c, hipMemcpyAsync(c->ubase + off, c->base_host.data() + off, n * sizeof(double), hipMemcpyHostToDevice,
                             c->stream), "upload boundary states");
    HIPCHK(c, hipMemcpyAsync(c->uin + off, c->ubase + off, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
           "upload boundary states");
    // the host copy must stay valid until the copy ran
    HIPCHK(c, hipStreamSynchronize(c->stream), "upload boundary states");
    return LBM_OK;
}

// After the boundary states changed: rebuild the synthetic-inflow generator
// (its mean field, sigma and u_ref follow them).
static int refresh_turbulence(lbm_ctx* c)
{
    if (!c->vk) return LBM_OK;
    VkGen* v = nullptr;
    std::string err;
    int rc = vk_create(&v, c->vkp, c->d.g, c->bits_host, c->base_host, err);
    if (rc != LBM_OK) return fail(c, rc, err);
    vk_destroy(c->vk);
    c->vk = v;
    return LBM_OK;
}

int lbm_set_inflow(lbm_ctx* c, int32_t face, const double* u)
{
    if (!c) return LBM_EINVAL;
    if (face < 0 || face > 5 || !u) return fail(c, LBM_EINVAL, "bad face or NULL profile");
    if (c->d.g.face[face] != LBM_INFLOW_EQ) return fail(c, LBM_EINVAL, "face is not an INFLOW_EQ face");
    const Geo& g = c->d.g;
    for (int i = 0; i < 3 * g.nz; i++)
        if (!std::isfinite(u[i])) return fail(c, LBM_EINVAL, "non-finite inflow velocity");
    // every cell of the face takes the profile at its height (the top row for z+)
    const int a = face >> 1;
    const long long n1 = a == 0 ? g.ny : g.nx, area = face_cells_host(g, face);
    double* dst = c->base_host.data() + 3 * (size_t)g.in_off[face];
    for (long long j = 0; j < area; j++) {
        const int z = a == 2 ? ((face & 1) ? g.nz - 1 : 0) : (int)(j / n1);
        for (int k = 0; k < 3; k++) dst[3 * j + k] = u[3 * z + k];
    }
    c->prof_set[face] = true;
    int rc = upload_base(c, face);
    if (rc != LBM_OK) return rc;
    return refresh_turbulence(c);
}

int lbm_set_inflow_face(lbm_ctx* c, int32_t face, const double* u)
{
    if (!c) return LBM_EINVAL;
    if (face < 0 || face > 5 || !u) return fail(c, LBM_EINVAL, "bad face or NULL boundary states");
    if (c->d.g.face[face] != LBM_INFLOW_EQ) return fail(c, LBM_EINVAL, "face is not an INFLOW_EQ face");
    const Geo& g = c->d.g;
    const long long n = 3 * face_cells_host(g, face);
    for (long long i = 0; i < n; i++)
        if (!std::isfinite(u[i])) return fail(c, LBM_EINVAL, "non-finite inflow velocity");
    std::copy(u, u + n, c->base_host.begin() + 3 * (size_t)g.in_off[face]);
    c->prof_set[face] = true;
    int rc = upload_base(c, face);
    if (rc != LBM_OK) return rc;
    return refresh_turbulence(c);
}

int lbm_set_rotation(lbm_ctx* c, const double* omega)
{
    if (!c) return LBM_EINVAL;
    if (!omega) return fail(c, LBM_EINVAL, "NULL rotation vector");
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(omega[a]) || std::fabs(omega[a]) > 0.25)
            return fail(c, LBM_EINVAL, "rotation component not finite or beyond 0.25 per time step");
    for (int a = 0; a < 3; a++) c->d.omega[a] = omega[a];
    return LBM_OK;
}

int lbm_earth_rotation(double latitude_deg, double dt_si, double grid_angle_deg, double* out)
{
    if (!out || !std::isfinite(latitude_deg) || !std::isfinite(dt_si) || !std::isfinite(grid_angle_deg) ||
        !(dt_si > 0.0) || std::fabs(latitude_deg) > 90.0)
        return fail(nullptr, LBM_EINVAL, "bad Earth rotation arguments");
    // east-north-up components of Omega dt, then onto the grid axes
    // ex = (cos a, sin a, 0), ey = (-sin a, cos a, 0) written in ENU
    const double kPi = 3.14159265358979323846;
    const double phi = latitude_deg * (kPi / 180.0), a = grid_angle_deg * (kPi / 180.0);
    const double w = LBM_OMEGA_EARTH * dt_si;
    const double north = w * std::cos(phi), up = w * std::sin(phi);
    out[0] = north * std::sin(a);   // (0, north, up) . ex
    out[1] = north * std::cos(a);   // (0, north, up) . ey
    out[2] = up;
    return LBM_OK;
}

int lbm_set_turbulence(lbm_ctx* c, const lbm_turbulence* p)
{
    if (!c) return LBM_EINVAL;
    if (p && has_halo(c)) return fail(c, LBM_ESTATE, "synthetic inflow on a slab (u_ref and e_c span all slabs)");
    VkGen* v = nullptr;
    if (p) {
        std::string err;
        int rc = vk_create(&v, *p, c->d.g, c->bits_host, c->base_host, err);
        if (rc != LBM_OK) return fail(c, rc, err);
    }
    // back to the boundary states everywhere; the generator writes its cells at the next step
    for (int F = 0; F < 6; F++) {
        int rc = upload_base(c, F);
        if (rc != LBM_OK) {
            vk_destroy(v);
            return rc;
        }
    }
    vk_destroy(c->vk);
    c->vk = v;
    if (p) c->vkp = *p;
    return LBM_OK;
}

int lbm_set_sponge(lbm_ctx* c, int32_t width, double strength)
{
    if (!c) return LBM_EINVAL;
    const Geo& g = c->d.g;
    const int lim = std::min(g.nx, std::min(g.ny, g.nz)) - 2;
    if (width < 0 || width > lim || !(strength >= 0.0 && strength <= 1.0))
        return fail(c, LBM_EINVAL, "sponge width outside [0, min(n) - 2] or strength outside [0, 1]");
    c->d.sponge_w = width;
    c->d.sponge_s = strength;
    return LBM_OK;
}

// Non-solid cells of the INFLOW_EQ faces, each on its owning face.
static int build_flux_cells(lbm_ctx* c)
{
    if (c->n_flux >= 0) return LBM_OK;
    const Geo& g = c->d.g;
    std::vector<int> sl, fc;
    for (int z = 0; z < g.nz; z++)
        for (int y = 0; y < g.ny; y++)
            for (int x = 0; x < g.nx; x++) {
                const int F = inflow_face_of(g, x, y, z);
                if (F < 0) continue;
                if ((c->bits_host[((size_t)y + (size_t)g.ny * z) * g.wpr + (x >> 6)] >> (x & 63)) & 1ull) continue;
                sl.push_back((int)inflow_slot(g, F, x, y, z));
                fc.push_back(F);
            }
    const long long n = (long long)sl.size();
    sl.insert(sl.end(), fc.begin(), fc.end());
    int rc;
    if ((rc = device_alloc(c, (void**)&c->flux_cells, sl.size() * sizeof(int), "flux cells")) != LBM_OK) return rc;
    if ((rc = device_alloc(c, (void**)&c->flux_red, (flux_partial_count() + 2) * sizeof(double), "flux sums")) !=
        LBM_OK)
        return rc;
    if (!sl.empty())
        HIPCHK(c, hipMemcpy(c->flux_cells, sl.data(), sl.size() * sizeof(int), hipMemcpyHostToDevice), "flux cells");
    c->n_flux = n;
    return LBM_OK;
}

// Net outward flux of the boundary states over the boundary cells.
static double base_flux(const lbm_ctx* c, long long* count)
{
    const Geo& g = c->d.g;
    double phi = 0.0;
    long long n = 0;
    for (int z = 0; z < g.nz; z++)
        for (int y = 0; y < g.ny; y++)
            for (int x = 0; x < g.nx; x++) {
                const int F = inflow_face_of(g, x, y, z);
                if (F < 0) continue;
                if ((c->bits_host[((size_t)y + (size_t)g.ny * z) * g.wpr + (x >> 6)] >> (x & 63)) & 1ull) continue;
                const double v = c->base_host[3 * (size_t)inflow_slot(g, F, x, y, z) + (F >> 1)];
                phi += (F & 1) ? v : -v;
                n++;
            }
    if (count) *count = n;
    return phi;
}

int lbm_net_flux(lbm_ctx* c, double* phi)
{
    if (!c) return LBM_EINVAL;
    if (!phi) return fail(c, LBM_EINVAL, "NULL output");
    int rc = build_flux_cells(c);
    if (rc != LBM_OK) return rc;
    *phi = 0.0;
    if (c->n_flux == 0) return LBM_OK;
    double* out = c->flux_red + flux_partial_count();
    HIPCHK(c, launch_flux_balance(c->flux_cells, c->flux_cells + c->n_flux, c->n_flux, c->uin, c->flux_red, out, 0,
                                  c->stream), "net flux");
    HIPCHK(c, hipMemcpyAsync(phi, out, sizeof(double), hipMemcpyDeviceToHost, c->stream), "net flux");
    HIPCHK(c, hipStreamSynchronize(c->stream), "net flux");
    return LBM_OK;
}

int lbm_balance_flux(lbm_ctx* c, int32_t mode, double* phi_before, double* phi_after)
{
    if (!c) return LBM_EINVAL;
    if (mode != 0 && has_halo(c)) return fail(c, LBM_ESTATE, "flux balancing on a slab (the flux spans all slabs)");
    if (mode < 0 || mode > 2) return fail(c, LBM_EINVAL, "flux balancing mode must be 0, 1 or 2");
    int rc = build_flux_cells(c);
    if (rc != LBM_OK) return rc;
    const Geo& g = c->d.g;
    if (mode == 0) {
        c->flux_mode = 0;
        if (phi_before && (rc = lbm_net_flux(c, phi_before)) != LBM_OK) return rc;
        if (phi_after) *phi_after = phi_before ? *phi_before : 0.0;
        return LBM_OK;
    }
    if (mode == 1) {
        long long n = 0;
        const double phi = base_flux(c, &n);
        if (phi_before) *phi_before = phi;
        if (n > 0) {
            // every entry of every INFLOW_EQ face moves by -(phi / n) n_out
            const double delta = phi / (double)n;
            for (int F = 0; F < 6; F++) {
                if (g.face[F] != LBM_INFLOW_EQ) continue;
                double* b = c->base_host.data() + 3 * (size_t)g.in_off[F];
                for (long long j = 0; j < face_cells_host(g, F); j++) b[3 * j + (F >> 1)] -= (F & 1) ? delta : -delta;
                if ((rc = upload_base(c, F)) != LBM_OK) return rc;
            }
            if ((rc = refresh_turbulence(c)) != LBM_OK) return rc;
        }
        if (phi_after) *phi_after = base_flux(c, nullptr);
        return LBM_OK;
    }
    // mode 2: balance the current field now, and before every step from now on
    c->flux_mode = 2;
    if (c->n_flux == 0) {
        if (phi_before) *phi_before = 0.0;
        if (phi_after) *phi_after = 0.0;
        return LBM_OK;
    }
    double* out = c->flux_red + flux_partial_count();
    double h[2];
    HIPCHK(c, launch_flux_balance(c->flux_cells, c->flux_cells + c->n_flux, c->n_flux, c->uin, c->flux_red, out, 1,
                                  c->stream), "flux balance");
    HIPCHK(c, launch_flux_balance(c->flux_cells, c->flux_cells + c->n_flux, c->n_flux, c->uin, c->flux_red, out + 1,
                                  0, c->stream), "net flux");
    HIPCHK(c, hipMemcpyAsync(h, out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "flux copy");
    HIPCHK(c, hipStreamSynchronize(c->stream), "flux copy");
    if (phi_before) *phi_before = h[0];
    if (phi_after) *phi_after = h[1];
    return LBM_OK;
}

int lbm_turbulence_info(lbm_ctx* c, int64_t* n_active, double* u_ref, double* e_c)
{
    if (!c) return LBM_EINVAL;
    vk_info(c->vk, n_active, u_ref, e_c);
    return LBM_OK;
}

int lbm_get_inflow(lbm_ctx* c, int32_t face, double* out)
{
    if (!c) return LBM_EINVAL;
    if (face < 0 || face > 5 || !out || c->d.g.in_off[face] < 0)
        return fail(c, LBM_EINVAL, "face is not an INFLOW_EQ face, or NULL output");
    const long long area = face_cells_host(c->d.g, face);
    HIPCHK(c, hipMemcpyAsync(out, c->uin + 3 * c->d.g.in_off[face], 3 * (size_t)area * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream), "copy inflow velocities");
    HIPCHK(c, hipStreamSynchronize(c->stream), "copy inflow velocities");
    return LBM_OK;
}

int lbm_reset(lbm_ctx* c, const double* u0)
{
    if (!c) return LBM_EINVAL;
    int rc = upload_u0(c, u0);
    if (rc != LBM_OK) return rc;
    HIPCHK(c, vk_apply(c->vk, c->uin, 0, c->stream), "synthetic inflow");
    HIPCHK(c, launch_init(c->d, c->u0, c->p.noise_amp, c->p.noise_seed, c->stream), "init kernel");
    c->phase = 0;
    c->t = 0;
    return LBM_OK;
}

static int check_ready(lbm_ctx* c)
{
    for (int F = 0; F < 6; F++)
        if (c->d.g.face[F] == LBM_INFLOW_EQ && !c->prof_set[F])
            return fail(c, LBM_ESTATE, "inflow face " + std::to_string(F) + " has no profile (lbm_set_inflow)");
    return LBM_OK;
}

static bool has_outflow(const lbm_ctx* c)
{
    for (int F = 0; F < 6; F++)
        if (c->d.g.face[F] == LBM_OUTFLOW_ZG) return true;
    return false;
}

static int mark(lbm_ctx* c)
{
    if (!c->profiling) return LBM_OK;
    if (c->ev_used == c->ev.size()) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e), "event create");
        c->ev.push_back(e);
    }
    HIPCHK(c, hipEventRecord(c->ev[c->ev_used++], c->stream), "event record");
    return LBM_OK;
}

static bool stats_due(const lbm_ctx* c)
{
    return c->stats && c->stats_stride > 0 && (c->t % c->stats_stride) == 0;
}

// One step t -> t+1.  probe_acc: NULL, or the probe accumulator to which the
// step kernels add u(t) of the probe cells (never together with stats).
static int one_step(lbm_ctx* c, void* probe_acc)
{
    void* st = stats_due(c) ? c->stats : nullptr;
    int rc;
    HIPCHK(c, vk_apply(c->vk, c->uin, c->t, c->stream), "synthetic inflow");
    if (c->flux_mode == 2)
        HIPCHK(c, launch_flux_balance(c->flux_cells, c->flux_cells + c->n_flux, c->n_flux, c->uin, c->flux_red,
                                      c->flux_red + flux_partial_count(), 1, c->stream), "flux balance");
    if (c->phase == 0) {
        if ((rc = mark(c)) != LBM_OK) return rc;
        HIPCHK(c, launch_step(c->d, 0, st, probe_acc, c->stream), "even step");
        if ((rc = mark(c)) != LBM_OK) return rc;
        c->phase = 1;
    } else {
        const bool out = has_outflow(c);
        if (out) HIPCHK(c, launch_outflow_ghost(c->d, c->stream), "outflow ghost");
        if ((rc = mark(c)) != LBM_OK) return rc;
        HIPCHK(c, launch_step(c->d, 1, st, probe_acc, c->stream), "odd step");
        if ((rc = mark(c)) != LBM_OK) return rc;
        if (out) HIPCHK(c, launch_outflow_copy(c->d, c->f, 0, c->stream), "outflow copy");
        c->phase = 0;
    }
    c->t += 1;
    return LBM_OK;
}

static int reduce(lbm_ctx* c, double out[5])
{
    HIPCHK(c, launch_mass(c->d, c->phase, c->red_partial, c->red_out, c->stream), "mass reduction");
    HIPCHK(c, hipMemcpyAsync(out, c->red_out, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "mass copy");
    HIPCHK(c, hipStreamSynchronize(c->stream), "mass sync");
    return LBM_OK;
}

static int watchdog(lbm_ctx* c)
{
    double r[5];
    int rc = reduce(c, r);
    if (rc != LBM_OK) return rc;
    if (r[4] != 0.0 || !std::isfinite(r[0]) || !std::isfinite(r[1]) || !(r[2] <= 0.25) || !(r[3] <= 0.5)) {
        char buf[200];
        snprintf(buf, sizeof buf, "unstable at t=%lld: max|u|^2=%g max|rho-rho0|=%g nonfinite=%g", (long long)c->t,
                 r[2], r[3], r[4]);
        return fail(c, LBM_EUNSTABLE, buf);
    }
    return LBM_OK;
}

static int step_n(lbm_ctx* c, int64_t n, void* acc)
{
    if (!c) return LBM_EINVAL;
    if (n < 0) return fail(c, LBM_EINVAL, "negative step count");
    if (acc && c->np == 0) return fail(c, LBM_ESTATE, "no probes registered");
    int rc = check_ready(c);
    if (rc != LBM_OK) return rc;
    const int wd = c->p.watchdog_stride;
    // The sample u(t+1) after step t is taken by the kernels of step t+1,
    // which form that velocity anyway (when lbm_set_probes found every probe
    // in their reach and that step collects no statistics); samples that no
    // step kernel takes (after the last step, before a watchdog check) go
    // through the probe kernel.  Both give the same bits.
    bool pending = false;   // u of the current state still to be added to acc
    for (int64_t k = 0; k < n; k++) {
        void* fold = nullptr;
        if (pending) {
            if (c->probe_fold && !stats_due(c)) fold = acc;
            else HIPCHK(c, launch_probe_cells(c->d, c->phase, c->probes, c->np, acc, c->stream), "probe accumulate");
            pending = false;
        }
        if ((rc = one_step(c, fold)) != LBM_OK) return rc;
        pending = acc != nullptr;
        if (wd > 0 && (c->t % wd) == 0) {
            if (pending) HIPCHK(c, launch_probe_cells(c->d, c->phase, c->probes, c->np, acc, c->stream), "probe accumulate");
            pending = false;
            if ((rc = watchdog(c)) != LBM_OK) return rc;
        }
    }
    if (pending) HIPCHK(c, launch_probe_cells(c->d, c->phase, c->probes, c->np, acc, c->stream), "probe accumulate");
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) { return step_n(c, n, nullptr); }

int lbm_step_probed(lbm_ctx* c, int64_t n, void* acc)
{
    if (!acc) return fail(c, LBM_EINVAL, "NULL accumulator");
    return step_n(c, n, acc);
}

int lbm_macros(lbm_ctx* c, void* rho, void* u, void* nut)
{
    if (!c) return LBM_EINVAL;
    if (!rho && !u && !nut) return LBM_OK;
    HIPCHK(c, launch_macros(c->d, c->phase, rho, u, nut, c->stream), "macros kernel");
    return LBM_OK;
}

int lbm_probe(lbm_ctx* c, const float* pts, int32_t np, float* out)
{
    if (!c) return LBM_EINVAL;
    if (np < 0 || (np > 0 && (!pts || !out))) return fail(c, LBM_EINVAL, "bad probe arguments");
    if (np == 0) return LBM_OK;
    for (int i = 0; i < 3 * np; i++)
        if (!std::isfinite(pts[i])) return fail(c, LBM_EINVAL, "non-finite probe coordinate");
    float* dbuf = nullptr;
    int rc = device_alloc(c, (void**)&dbuf, (size_t)np * 7 * sizeof(float), "probe buffer");
    if (rc != LBM_OK) return rc;
    hipError_t e = hipMemcpyAsync(dbuf, pts, (size_t)np * 3 * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_probe_points(c->d, c->phase, dbuf, np, dbuf + 3 * (size_t)np, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dbuf + 3 * (size_t)np, (size_t)np * 4 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dbuf);
    if (e != hipSuccess) return hip_fail(c, e, "probe");
    return LBM_OK;
}

int lbm_probe_noalloc(lbm_ctx* c, const float* pts, int32_t np, float* out)
{
    if (!c) return LBM_EINVAL;
    if (np < 0 || (np > 0 && (!pts || !out))) return fail(c, LBM_EINVAL, "bad probe arguments");
    if (np > LBM_PROBE_NOALLOC_MAX)
        return fail(c, LBM_EINVAL, "np = " + std::to_string(np) + " exceeds LBM_PROBE_NOALLOC_MAX (" +
                                       std::to_string(LBM_PROBE_NOALLOC_MAX) + ")");
    if (np == 0) return LBM_OK;
    for (int i = 0; i < 3 * np; i++)
        if (!std::isfinite(pts[i])) return fail(c, LBM_EINVAL, "non-finite probe coordinate");
    float* dbuf;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        dbuf = g_scratch[c->device];
    }
    if (!dbuf) return fail(c, LBM_ESTATE, "no scratch address for this device");
    // points in, results out: every value the kernel reads is written first
    hipError_t e = hipMemcpyAsync(dbuf, pts, (size_t)np * 3 * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_probe_points(c->d, c->phase, dbuf, np, dbuf + 3 * (size_t)np, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dbuf + 3 * (size_t)np, (size_t)np * 4 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "probe (no allocation)");
    return LBM_OK;
}

int lbm_mass(lbm_ctx* c, double* mass, double* energy)
{
    if (!c) return LBM_EINVAL;
    double r[5];
    int rc = reduce(c, r);
    if (rc != LBM_OK) return rc;
    if (mass) *mass = (double)c->interior * c->p.rho0 + r[0];
    if (energy) *energy = r[1];
    return LBM_OK;
}

int lbm_get_state(lbm_ctx* c, void* dst, int64_t* t)
{
    if (!c) return LBM_EINVAL;
    if (!dst) return fail(c, LBM_EINVAL, "NULL destination");
    HIPCHK(c, launch_export(c->d, c->phase, dst, c->stream), "export kernel");
    if (t) *t = c->t;
    return LBM_OK;
}

int lbm_set_state(lbm_ctx* c, const void* src, int64_t t)
{
    if (!c) return LBM_EINVAL;
    if (!src || t < 0) return fail(c, LBM_EINVAL, "NULL source or negative time");
    HIPCHK(c, launch_import(c->d, src, c->stream), "import kernel");
    c->phase = 0;
    c->t = t;
    // with the watchdog on, a corrupt state (non-finite or out-of-range
    // values) is reported at once instead of at the next check
    if (c->p.watchdog_stride > 0) return watchdog(c);
    return LBM_OK;
}

int lbm_set_probes(lbm_ctx* c, const int32_t* cells, int32_t np)
{
    if (!c) return LBM_EINVAL;
    if (np < 0 || np > 4096 || (np > 0 && !cells)) return fail(c, LBM_EINVAL, "bad probe list");
    const Geo& g = c->d.g;
    for (int p = 0; p < np; p++) {
        const int x = cells[3 * p], y = cells[3 * p + 1], z = cells[3 * p + 2];
        if (x < 0 || y < 0 || z < 0 || x >= g.nx || y >= g.ny || z >= g.nz)
            return fail(c, LBM_EINVAL, "probe cell outside the grid");
    }
    if (c->probes || c->probe_tab) {
        HIPCHK(c, hipStreamSynchronize(c->stream), "probe sync");
        if (c->probes) (void)hipFree(c->probes);
        if (c->probe_tab) (void)hipFree(c->probe_tab);
        c->probes = nullptr;
        c->probe_tab = nullptr;
    }
    c->np = 0;
    c->probe_fold = false;
    c->d.probes = AdjProbes{nullptr, nullptr, nullptr, 0, nullptr};
    if (np == 0) return LBM_OK;
    int rc = device_alloc(c, (void**)&c->probes, (size_t)np * 3 * sizeof(int), "probes");
    if (rc != LBM_OK) return rc;
    HIPCHK(c, hipMemcpy(c->probes, cells, (size_t)np * 3 * sizeof(int), hipMemcpyHostToDevice), "probe upload");
    // adjoint probe table: one bit per 64-cell chunk of a row, then the
    // (cell, probe) entries sorted by cell and, within a cell, by probe
    const long long nchunks = (long long)g.ncx * g.ny * g.nz;
    const size_t nwords = (size_t)((nchunks + 31) / 32);
    std::vector<std::pair<unsigned, int>> ent((size_t)np);
    for (int p = 0; p < np; p++)
        ent[(size_t)p] = {(unsigned)(cells[3 * p] + (long long)g.nx * (cells[3 * p + 1] + (long long)g.ny * cells[3 * p + 2])), p};
    std::sort(ent.begin(), ent.end());
    std::vector<uint32_t> bits(nwords, 0u);
    std::vector<unsigned> pc((size_t)np);
    std::vector<int> pid((size_t)np);
    for (size_t e = 0; e < ent.size(); e++) {
        pc[e] = ent[e].first;
        pid[e] = ent[e].second;
        const long long row = (long long)ent[e].first / g.nx;
        const long long chunk = (long long)(ent[e].first % g.nx) / 64 + (long long)g.ncx * row;
        bits[(size_t)(chunk >> 5)] |= 1u << (chunk & 31);
    }
    const size_t bytes = nwords * 4 + (size_t)np * 8;
    rc = device_alloc(c, &c->probe_tab, bytes, "probe table");
    if (rc != LBM_OK) return rc;
    auto* tb = (char*)c->probe_tab;
    HIPCHK(c, hipMemcpy(tb, bits.data(), nwords * 4, hipMemcpyHostToDevice), "probe table upload");
    HIPCHK(c, hipMemcpy(tb + nwords * 4, pc.data(), (size_t)np * 4, hipMemcpyHostToDevice), "probe table upload");
    HIPCHK(c, hipMemcpy(tb + nwords * 4 + (size_t)np * 4, pid.data(), (size_t)np * 4, hipMemcpyHostToDevice),
           "probe table upload");
    c->d.probes = AdjProbes{(const uint32_t*)tb, (const unsigned*)(tb + nwords * 4),
                            (const int*)(tb + nwords * 4 + (size_t)np * 4), np, nullptr};
    c->np = np;
    // The step kernels can take the probe samples when every probe cell is a
    // fluid, non-inflow cell off the x faces whose odd-step wave the fast
    // kernel runs (not the general per-cell path); the even kernel runs all.
    bool fold = true;
    for (int p = 0; p < np && fold; p++) {
        const int x = cells[3 * p], y = cells[3 * p + 1], z = cells[3 * p + 2];
        const bool solid = (c->bits_host[((size_t)y + (size_t)g.ny * z) * g.wpr + (x >> 6)] >> (x & 63)) & 1ull;
        fold = !solid && inflow_face_of(g, x, y, z) < 0 && x >= 1 && x <= g.nx - 2 &&
               !odd_wave_is_general(g, x >> 6, y, z);
    }
    c->probe_fold = fold;
    return LBM_OK;
}

int lbm_probe_accumulate(lbm_ctx* c, void* acc)
{
    if (!c) return LBM_EINVAL;
    if (!acc) return fail(c, LBM_EINVAL, "NULL accumulator");
    if (c->np == 0) return fail(c, LBM_ESTATE, "no probes registered");
    HIPCHK(c, launch_probe_cells(c->d, c->phase, c->probes, c->np, acc, c->stream), "probe accumulate");
    return LBM_OK;
}

int lbm_set_stats(lbm_ctx* c, void* acc, int32_t stride)
{
    if (!c) return LBM_EINVAL;
    if (!acc || stride <= 0) {
        c->stats = nullptr;
        c->stats_stride = 0;
        return LBM_OK;
    }
    c->stats = acc;
    c->stats_stride = stride;
    return LBM_OK;
}

int lbm_push_step(lbm_ctx* c, const void* src, void* dst)
{
    if (!c) return LBM_EINVAL;
    if (has_halo(c)) return fail(c, LBM_ESTATE, "push step on a slab");
    if (!src || !dst || src == dst) return fail(c, LBM_EINVAL, "src and dst must be distinct device arrays");
    if (c->vk) return fail(c, LBM_ESTATE, "push step with synthetic inflow turbulence on");
    // the push kernel addresses the two candidate slots of a direction in the
    // canonical arrays with 32-bit byte offsets (slot_span slices apart at most)
    if (slot_span(c->d.g.face) * c->d.g.N * (long long)c->store_bytes >= (1ll << 32))
        return fail(c, LBM_EINVAL, "grid too large for the push step (a canonical slice must stay below " +
                                       std::string(slot_span(c->d.g.face) == 2 ? "2 GiB" : "512 MiB with free-slip y or z faces") + ")");
    int rc = check_ready(c);
    if (rc != LBM_OK) return rc;
    HIPCHK(c, launch_push(c->d, src, dst, c->stream), "push step");
    return LBM_OK;
}

int lbm_adjoint_step(lbm_ctx* c, const void* f_t, const void* lam_next, void* lam, const void* probe_src,
                     void* g_inflow)
{
    if (!c) return LBM_EINVAL;
    if (has_halo(c)) return fail(c, LBM_ESTATE, "adjoint step on a slab");
    if (!f_t || !lam_next || !lam || lam == lam_next) return fail(c, LBM_EINVAL, "bad adjoint arguments");
    {
        // the adjoint kernels address the two candidate slots of a direction
        // with 32-bit byte offsets (slot_span adjoint slices apart at most)
        const long long real_bytes = c->p.storage == LBM_F64 ? 8 : 4;
        if (slot_span(c->d.g.face) * c->d.g.N * real_bytes >= (1ll << 32))
            return fail(c, LBM_EINVAL, "grid too large for the adjoint (an adjoint slice must stay below " +
                                           std::string(slot_span(c->d.g.face) == 2 ? "2 GiB" : "512 MiB with free-slip y or z faces") + ")");
    }
    if (probe_src && c->np == 0) return fail(c, LBM_ESTATE, "probe source without registered probes");
    if (c->vk) return fail(c, LBM_ESTATE, "adjoint step with synthetic inflow turbulence on");
    if (c->d.sponge_w > 0 && c->d.sponge_s > 0.0) return fail(c, LBM_ESTATE, "adjoint step with the sponge on");
    int rc = check_ready(c);
    if (rc != LBM_OK) return rc;
    HIPCHK(c, launch_adjoint(c->d, f_t, lam_next, lam, probe_src, g_inflow, c->stream), "adjoint step");
    return LBM_OK;
}

int lbm_voxelize(const lbm_grid* grid, const double* tri, int32_t nt, const int32_t* starts, int32_t nm,
                 int32_t passes, uint8_t* solid)
{
    std::string err;
    const int rc = voxelize(grid, tri, nt, starts, nm, passes, solid, err);
    if (rc != LBM_OK) return fail(nullptr, rc, err);
    return LBM_OK;
}

int lbm_halo_pack(lbm_ctx* c, int32_t side, void* buf)
{
    if (!c) return LBM_EINVAL;
    if (side < 0 || side > 1 || !c->halo[2 + side] || !buf)
        return fail(c, LBM_EINVAL, "side is not a HALO face, or NULL buffer");
    HIPCHK(c, launch_halo(c->d, side, c->phase, 0, buf, c->stream), "halo pack");
    return LBM_OK;
}

int lbm_halo_unpack(lbm_ctx* c, int32_t side, const void* buf)
{
    if (!c) return LBM_EINVAL;
    if (side < 0 || side > 1 || !c->halo[2 + side] || !buf)
        return fail(c, LBM_EINVAL, "side is not a HALO face, or NULL buffer");
    HIPCHK(c, launch_halo(c->d, side, c->phase, 1, const_cast<void*>(buf), c->stream), "halo unpack");
    return LBM_OK;
}

int lbm_profile(lbm_ctx* c, int32_t enable)
{
    if (!c) return LBM_EINVAL;
    c->profiling = enable != 0;
    c->ev_used = 0;
    return LBM_OK;
}

int lbm_profile_read(lbm_ctx* c, double* total_ms, int64_t* launches)
{
    if (!c) return LBM_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream), "profile sync");
    double tot = 0.0;
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]), "event elapsed");
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)(c->ev_used / 2);
    c->ev_used = 0;
    return LBM_OK;
}

}  // extern "C"
