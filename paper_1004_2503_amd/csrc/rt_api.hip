// rt_api.hip -- host side of the C ABI declared in include/rt.h.
//
// The host only validates, drives and reads back (Appendix A: the host sends
// the device one signal per step and never computes on the fields).  Every
// argument check happens before the first HIP call, so invalid input is
// rejected without touching the device.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mlp_device.h"

using namespace rtk;

namespace {

constexpr double KB = 1.380649e-16;
constexpr double EV = 1.602176634e-12;
constexpr double E_ION_EV = 13.6;
constexpr int MAX_NSUB = 4096;
#ifndef RT_M1_ZC
#define RT_M1_ZC 64
#endif
#ifndef RT_M1_ZC_MIN
#define RT_M1_ZC_MIN 16
#endif
#ifndef RT_M1_ZC_BLOCKS
#define RT_M1_ZC_BLOCKS 2048
#endif
constexpr int ZC_DEFAULT = RT_M1_ZC;  // planes per block along z (the longest chunk)
constexpr int ZC_MIN = RT_M1_ZC_MIN;  // shortest chunk the grid size may ask for
// chunks are halved (down to ZC_MIN) while a grid has fewer 64 x TY tiles
// than this, so that small and mid-size grids still fill the chip
constexpr int ZC_BLOCKS = RT_M1_ZC_BLOCKS;
constexpr int ZC_LONG = 128;           // chunk of the largest grids
constexpr int ZC_LONG_BLOCKS = 8192;   // 64 x TY_LF tiles x chunks needed for it
#ifndef RT_M1_BIG_MIN
#define RT_M1_BIG_MIN 1024
#endif
constexpr int BIG_MIN_BLOCKS = RT_M1_BIG_MIN;   // 64 x TY_LF tiles from this many on
static_assert(ZC_MIN >= 2 && ZC_MIN <= ZC_DEFAULT, "z chunk bounds");
constexpr double SIGMA_T = 6.6524587321e-25;  // Thomson cross-section [cm^2]
constexpr int HSUM_DOUBLES = 256 + 2 * 257;   // histogram sums + edges

struct Ev {
    hipEvent_t a, b;
};

}  // namespace

// Tiles of one form of the step and the point sources binned into them.
struct TileSet {
    int ty = 0, nty = 0, nblocks = 0;
    int zc = 0, nzc = 0;            // planes per z chunk, chunks
    int32_t *d_src_ptr = nullptr;   // per tile [start, end) into key/rate
    int32_t *d_src_key = nullptr;
    float *d_src_rate = nullptr;
};

struct rt_ctx {
    rt_params p;
    rt_fields f;
    hipStream_t stream = nullptr;
    int cur = 0;
    int ntx = 0;
    uint32_t ncell = 0;
    // 0: LF forms on large grids (TY_LF rows), 1: LF forms on small grids
    // (TY rows), 2: the HLL form (TY_HLL rows)
    TileSet geo[3];
    // the current source set on the host; each tile set's lists are built
    // when a step first needs them
    std::vector<int32_t> src_ijk;
    std::vector<double> src_ndot;
    bool geo_ready[3] = {true, true, true};   // the empty set at rt_init
    int64_t nsrc = 0;
    double ndot_total = 0.0;
    double *d_part = nullptr;
    int npart = 0;
    double *d_fin = nullptr;   // first-level finalisation rows
    uint64_t *d_mask = nullptr;   // FP64 cells left by the step (mixed forms)
    uint64_t *d_gmask = nullptr;  // groups of 64 mask words holding a marked cell
    uint32_t *d_goff = nullptr;   // marked cells per group -> offsets (deferred kernels)
    uint32_t *d_cells = nullptr;  // dense list of the marked cells (one slot per cell)
    uint64_t *d_mask2 = nullptr;  // the learned form's rejected cells
    uint64_t nwords = 0;
    int gwords = 0;               // 64-bit words of d_gmask
    int nb2 = 0;                  // blocks of the deferred FP64 chemistry
    double *d_acc = nullptr;
    float *d_sink = nullptr;
    unsigned long long *d_hcount = nullptr;  // RT_HIST_MAX_BINS
    double *d_hsum = nullptr;                // 256 + edges 2 * 257
    unsigned long long *d_hlimb = nullptr;   // exact histogram sums: 256 bins of limbs
    double t = 0.0, emitted = 0.0, photons_initial = 0.0, nh_sum = 0.0;
    int64_t steps = 0;
    int64_t hist_host[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool prof = false;
    std::vector<Ev> ev;
    size_t ev_used = 0;
    // learned chemistry
    bool surr = false;
    __bf16 *d_surr_pk = nullptr;
    float *d_surr_bias = nullptr;
    float surr_norm[SURR_NNORM] = {};
    float surr_tol = 0.0f;
    // expansion rate H [1/s] of the steps that follow (0: static)
    double hubble = 0.0;
};

static int check_params(const rt_params *p)
{
    if (!p) return RT_E_ARG;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return RT_E_ARG;
    const double ncell = double(p->nx) * double(p->ny) * double(p->nz);
    if (ncell >= 4294967296.0) return RT_E_ARG;
    for (int f = 0; f < 6; ++f)
        if (p->bc[f] < RT_BC_PERIODIC || p->bc[f] > RT_BC_REFLECT) return RT_E_ARG;
    for (int d = 0; d < 3; ++d)
        if ((p->bc[2 * d] == RT_BC_PERIODIC) != (p->bc[2 * d + 1] == RT_BC_PERIODIC))
            return RT_E_ARG;
    if (p->chem < RT_CHEM_FULL || p->chem > RT_CHEM_FROZEN) return RT_E_ARG;
    if (p->prec != RT_PREC_FP32 && p->prec != RT_PREC_MIXED) return RT_E_ARG;
    if (p->sub != RT_SUB_FIXED && p->sub != RT_SUB_ADAPTIVE) return RT_E_ARG;
    if (check_clump(*p) != RT_OK) return RT_E_ARG;
    if (p->flux != RT_FLUX_LF && p->flux != RT_FLUX_HLL) return RT_E_ARG;
    if (!(p->dx_cm > 0.0) || !isfinite(p->dx_cm)) return RT_E_ARG;
    if (!(p->c_cms > 0.0) || !isfinite(p->c_cms)) return RT_E_ARG;
    if (!(p->sigma_n > 0.0) || !(p->sigma_e > 0.0) || !(p->egamma_eV > 0.0)) return RT_E_ARG;
    if (!(p->T_floor >= 0.0) || !isfinite(p->T_floor)) return RT_E_ARG;
    if (p->sub == RT_SUB_ADAPTIVE && !(p->sub_eps > 0.0 && p->sub_eps <= 1.0)) return RT_E_ARG;
    if (!(p->xhi_fp64_thr >= 0.0 && p->xhi_fp64_thr <= 1.0)) return RT_E_ARG;
    return RT_OK;
}

static int check_fields(const rt_fields *f)
{
    if (!f) return RT_E_ARG;
    const void *ptrs[11] = {f->N[0], f->N[1], f->Fx[0], f->Fx[1], f->Fy[0], f->Fy[1],
                            f->Fz[0], f->Fz[1], f->xHI, f->T, f->nH};
    for (int i = 0; i < 11; ++i) {
        if (!ptrs[i]) return RT_E_ARG;
        for (int j = 0; j < i; ++j)
            if (ptrs[i] == ptrs[j]) return RT_E_ARG;
    }
    return RT_OK;
}

static void free_ctx(rt_ctx *c)
{
    if (!c) return;
    for (TileSet &g : c->geo) {
        if (g.d_src_ptr) (void)hipFree(g.d_src_ptr);
        if (g.d_src_key) (void)hipFree(g.d_src_key);
        if (g.d_src_rate) (void)hipFree(g.d_src_rate);
    }
    if (c->d_part) (void)hipFree(c->d_part);
    if (c->d_fin) (void)hipFree(c->d_fin);
    if (c->d_mask) (void)hipFree(c->d_mask);
    if (c->d_gmask) (void)hipFree(c->d_gmask);
    if (c->d_goff) (void)hipFree(c->d_goff);
    if (c->d_cells) (void)hipFree(c->d_cells);
    if (c->d_mask2) (void)hipFree(c->d_mask2);
    if (c->d_acc) (void)hipFree(c->d_acc);
    if (c->d_sink) (void)hipFree(c->d_sink);
    if (c->d_hcount) (void)hipFree(c->d_hcount);
    if (c->d_hsum) (void)hipFree(c->d_hsum);
    if (c->d_hlimb) (void)hipFree(c->d_hlimb);
    if (c->d_surr_pk) (void)hipFree(c->d_surr_pk);
    if (c->d_surr_bias) (void)hipFree(c->d_surr_bias);
    for (auto &e : c->ev) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    delete c;
}

extern "C" const char *rt_strerror(int code)
{
    switch (code) {
    case RT_OK: return "ok";
    case RT_E_ARG: return "invalid argument";
    case RT_E_CFL: return "time step above the light-crossing bound dx/(3c)";
    case RT_E_STATE: return "invalid call order or null context";
    case RT_E_HIP: return "HIP runtime failure";
    case RT_E_NONFINITE: return "a step produced a non-finite value";
    case RT_E_NOMEM: return "device allocation failed";
    case RT_E_SCRATCH: return "request exceeds the fixed scratch of an allocation-free entry point";
    default: return "unknown error";
    }
}

// Planes per block along z: the longest chunk (at most the grid's depth),
// halved while the grid has fewer than ZC_BLOCKS tiles of 64 x ty cells.
// Each block marches its chunk serially, so on small grids long chunks
// leave most compute units idle; short chunks re-read more z-halo planes
// (two per chunk), which the large grids avoid.
static int z_chunk(int ntx, int ny, int nz, int ty)
{
    // the largest grids take 128-plane chunks as long as they still have
    // ZC_LONG_BLOCKS of them (32 per compute unit): fewer z-halo planes,
    // while enough blocks remain to even out the end of the launch.
    // Measured: 1024^3 12.16 against 12.22 ms with 64 planes; 512^3, which
    // would have 1024 such blocks, 1.745 against 1.689 ms.
    const int64_t layer = int64_t(ntx) * ((ny + TY_LF - 1) / TY_LF);
    if (nz >= ZC_LONG && layer * ((nz + ZC_LONG - 1) / ZC_LONG) >= ZC_LONG_BLOCKS)
        return ZC_LONG;
    int zc = std::min(ZC_DEFAULT, nz);
    const int64_t cols = int64_t(ntx) * ((ny + ty - 1) / ty);
    while (zc / 2 >= ZC_MIN && cols * ((nz + zc - 1) / zc) < ZC_BLOCKS) zc /= 2;
    return zc;
}

// The deferred-cell mask (written whole by every step that uses it) and its
// group bits (set by the step, cleared by the finalisation; zero to start).
static int alloc_masks(rt_ctx *c)
{
    if (!c->d_mask && hipMalloc(&c->d_mask, c->nwords * sizeof(uint64_t)) != hipSuccess) {
        (void)hipGetLastError();
        return RT_E_NOMEM;
    }
    if (!c->d_goff &&
        hipMalloc(&c->d_goff, defer_offsets_size(c->nwords) * sizeof(uint32_t)) !=
            hipSuccess) {
        (void)hipGetLastError();
        return RT_E_NOMEM;
    }
    if (!c->d_cells && hipMalloc(&c->d_cells, size_t(c->ncell) * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return RT_E_NOMEM;
    }
    if (!c->d_gmask) {
        if (hipMalloc(&c->d_gmask, size_t(c->gwords) * sizeof(uint64_t)) != hipSuccess) {
            (void)hipGetLastError();
            return RT_E_NOMEM;
        }
        if (hipMemsetAsync(c->d_gmask, 0, size_t(c->gwords) * sizeof(uint64_t), c->stream) !=
            hipSuccess)
            return RT_E_HIP;
    }
    return RT_OK;
}

extern "C" int rt_init(const rt_params *params, const rt_fields *fields, void *hip_stream,
                       rt_ctx **out)
{
    if (!out) return RT_E_ARG;
    *out = nullptr;
    int rc = check_params(params);
    if (rc != RT_OK) return rc;
    rc = check_fields(fields);
    if (rc != RT_OK) return rc;

    rt_ctx *c = new (std::nothrow) rt_ctx();
    if (!c) return RT_E_NOMEM;
    c->p = *params;
    c->f = *fields;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ncell = uint32_t(params->nx) * uint32_t(params->ny) * uint32_t(params->nz);
    c->ntx = (params->nx + TX - 1) / TX;
    for (int gi = 0; gi < 3; ++gi) {
        TileSet &g = c->geo[gi];
        g.ty = gi == 0 ? TY_LF : (gi == 1 ? TY : TY_HLL);
        g.nty = (params->ny + g.ty - 1) / g.ty;
        // both LF tile sets chunk z as the small tiles need
        g.zc = z_chunk(c->ntx, params->ny, params->nz, gi == 2 ? TY_HLL : TY);
        g.nzc = (params->nz + g.zc - 1) / g.zc;
        const int64_t nb = int64_t(c->ntx) * g.nty * g.nzc;
        if (nb > (int64_t(1) << 30)) {
            delete c;
            return RT_E_ARG;
        }
        g.nblocks = int(nb);
    }
    // the deferred chemistry's mask: needed by the mixed and adaptive forms
    // from the start, by the learned chemistry once it is switched on
    const bool defer = params->prec == RT_PREC_MIXED || params->sub == RT_SUB_ADAPTIVE;
    c->nwords = uint64_t(params->nz) * uint64_t(params->ny) * uint64_t(c->ntx);
    c->nb2 = defer_chem_blocks(c->nwords);
    c->gwords = int((mask_groups(c->nwords) + 63) / 64);
    // partial rows: a step writes one per block of whichever tile set it
    // runs on, then the deferred chemistry nb2 more after them
    c->npart = std::max(std::max(std::max(c->geo[0].nblocks, c->geo[1].nblocks),
                                 c->geo[2].nblocks) + 2 * c->nb2,
                        std::max(state_sums_blocks(c->ncell),
                                 (2 * plateau_blocks(c->ncell) + NRED - 1) / NRED));
    if (defer) {
        rc = alloc_masks(c);
        if (rc != RT_OK) {
            free_ctx(c);
            return rc;
        }
    }

    if (hipMalloc(&c->d_part, size_t(c->npart) * NRED * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_fin, size_t(FIN1_BLOCKS) * NRED * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_acc, ACC_SIZE * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->geo[0].d_src_ptr, size_t(c->geo[0].nblocks + 1) * sizeof(int32_t)) !=
            hipSuccess ||
        hipMalloc(&c->geo[1].d_src_ptr, size_t(c->geo[1].nblocks + 1) * sizeof(int32_t)) !=
            hipSuccess ||
        hipMalloc(&c->geo[2].d_src_ptr, size_t(c->geo[2].nblocks + 1) * sizeof(int32_t)) !=
            hipSuccess ||
        hipMalloc(&c->d_sink, NTHREADS_MAX * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->d_hcount, RT_HIST_MAX_BINS * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->d_hsum, HSUM_DOUBLES * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_hlimb, hist_limb_count(256) * sizeof(unsigned long long)) !=
            hipSuccess) {
        (void)hipGetLastError();
        free_ctx(c);
        return RT_E_NOMEM;
    }
    if (hipMemsetAsync(c->geo[0].d_src_ptr, 0, size_t(c->geo[0].nblocks + 1) * sizeof(int32_t),
                       c->stream) != hipSuccess ||
        hipMemsetAsync(c->geo[1].d_src_ptr, 0, size_t(c->geo[1].nblocks + 1) * sizeof(int32_t),
                       c->stream) != hipSuccess ||
        hipMemsetAsync(c->geo[2].d_src_ptr, 0, size_t(c->geo[2].nblocks + 1) * sizeof(int32_t),
                       c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_acc, 0, ACC_SIZE * sizeof(double), c->stream) != hipSuccess) {
        free_ctx(c);
        return RT_E_HIP;
    }
    // sums of the initial state (photons_initial and the averages before
    // any step)
    const int nsb = state_sums_blocks(c->ncell);
    if (launch_state_sums(fields->N[0], fields->xHI, fields->nH, c->ncell, c->d_part, nsb,
                          c->stream) != hipSuccess ||
        launch_finalize(c->d_part, nsb, c->d_fin, c->d_acc, 1, 0.0, 0.0, c->stream) !=
            hipSuccess) {
        free_ctx(c);
        return RT_E_HIP;
    }
    double acc[ACC_SIZE];
    if (hipMemcpyAsync(acc, c->d_acc, sizeof(acc), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        free_ctx(c);
        return RT_E_HIP;
    }
    const double vol = params->dx_cm * params->dx_cm * params->dx_cm;
    c->photons_initial = acc[ACC_CUR + R_N] * vol;
    c->nh_sum = acc[ACC_CUR + R_NH];
    *out = c;
    return RT_OK;
}

extern "C" int rt_inject_sources(rt_ctx *c, int64_t n, const int32_t *ijk, const double *ndot)
{
    if (!c) return RT_E_STATE;
    if (n < 0 || n > (int64_t(1) << 31) - 1) return RT_E_ARG;
    if (n > 0 && (!ijk || !ndot)) return RT_E_ARG;
    return rtk::inject_host(c, n, ijk, ndot);
}

extern "C" int rt_sources_from_particles(rt_ctx *c, int64_t n, const double *pos,
                                         const double *age_next, const double *lifetime,
                                         const double *q_per_baryon, const double *mass_g,
                                         double t_p, double t_next, double f_esc, double a_b,
                                         double k_b, int64_t *n_active)
{
    if (!c) return RT_E_STATE;
    if (n < 0 || n > (int64_t(1) << 31) - 1) return RT_E_ARG;
    if (n > 0 && (!pos || !age_next || !lifetime || !q_per_baryon || !mass_g)) return RT_E_ARG;
    if (!(t_p > 0.0) || !(t_next > t_p) || !isfinite(t_next)) return RT_E_ARG;
    if (!(f_esc >= 0.0 && f_esc <= 1.0)) return RT_E_ARG;
    if (!(a_b >= 0.0) || !isfinite(a_b) || !(k_b >= 0.0) || !isfinite(k_b)) return RT_E_ARG;
    // boost factor at the middle of the interval (libm exp, as on any host)
    const double t_mid = 0.5 * (t_p + t_next);
    const double boost = fmax(1.0, a_b * exp(k_b / t_mid));
    if (!isfinite(boost)) return RT_E_ARG;
    if (n == 0) {
        if (n_active) *n_active = 0;
        return inject_host(c, 0, nullptr, nullptr);
    }
    int32_t *d_ijk = nullptr, *d_bad = nullptr;
    double *d_rate = nullptr;
    if (hipMalloc(&d_ijk, size_t(n) * 3 * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&d_rate, size_t(n) * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_bad, sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        if (d_ijk) (void)hipFree(d_ijk);
        if (d_rate) (void)hipFree(d_rate);
        return RT_E_NOMEM;
    }
    std::vector<int32_t> ijk(static_cast<size_t>(n) * 3);
    std::vector<double> rate(static_cast<size_t>(n));
    int32_t bad = 0;
    const rt_params &p = c->p;
    int rc = RT_OK;
    if (hipMemsetAsync(d_bad, 0, sizeof(int32_t), c->stream) != hipSuccess ||
        launch_particle_rates(n, pos, age_next, lifetime, q_per_baryon, mass_g, t_next - t_p,
                              f_esc, boost, p.dx_cm, p.nx, p.ny, p.nz, d_ijk, d_rate, d_bad,
                              c->stream) != hipSuccess ||
        hipMemcpyAsync(ijk.data(), d_ijk, ijk.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess ||
        hipMemcpyAsync(rate.data(), d_rate, rate.size() * sizeof(double),
                       hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        rc = RT_E_HIP;
    (void)hipFree(d_ijk);
    (void)hipFree(d_rate);
    (void)hipFree(d_bad);
    if (rc != RT_OK) return rc;
    if (bad) return RT_E_ARG;   // the old source set stays
    // emitting particles, in particle order
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (rate[size_t(i)] > 0.0) {
            ijk[size_t(3 * m)] = ijk[size_t(3 * i)];
            ijk[size_t(3 * m + 1)] = ijk[size_t(3 * i + 1)];
            ijk[size_t(3 * m + 2)] = ijk[size_t(3 * i + 2)];
            rate[size_t(m)] = rate[size_t(i)];
            ++m;
        }
    }
    if (n_active) *n_active = m;
    return inject_host(c, m, ijk.data(), rate.data());
}

// Bin host sources into the per-tile lists of both tile sets (duplicate
// cells summed in input order) and replace the context's source set.
namespace {
struct Lists {
    std::vector<int32_t> ptr, key;
    std::vector<float> rate;
};

Lists bin_sources(const rt_ctx *c, const TileSet &g, int64_t n, const int32_t *ijk,
                  const double *ndot)
{
    const rt_params &p = c->p;
    const int nt = TX * g.ty;
    struct Src {
        int32_t tile, key;
        double ndot;
    };
    // two stable counting sorts (by cell within the tile, then by tile) give
    // the (tile, cell) order with equal cells kept in input order, so
    // duplicates are summed in input order
    const int64_t nkeys = int64_t(g.zc) * nt;
    std::vector<int32_t> tile_of(static_cast<size_t>(n)), key_of(static_cast<size_t>(n));
    std::vector<int64_t> kcount(static_cast<size_t>(nkeys) + 1, 0);
    std::vector<int64_t> tcount(static_cast<size_t>(g.nblocks) + 1, 0);
    for (int64_t s = 0; s < n; ++s) {
        const int32_t i = ijk[3 * s], j = ijk[3 * s + 1], k = ijk[3 * s + 2];
        const int itx = i / TX, ity = j / g.ty, izc = k / g.zc;
        const int tile = (izc * g.nty + ity) * c->ntx + itx;
        const int key = (k - izc * g.zc) * nt + (j - ity * g.ty) * TX + (i - itx * TX);
        tile_of[size_t(s)] = tile;
        key_of[size_t(s)] = key;
        kcount[size_t(key) + 1] += 1;
        tcount[size_t(tile) + 1] += 1;
    }
    for (int64_t q = 0; q < nkeys; ++q) kcount[size_t(q) + 1] += kcount[size_t(q)];
    for (int b = 0; b < g.nblocks; ++b) tcount[size_t(b) + 1] += tcount[size_t(b)];
    std::vector<int64_t> by_key(static_cast<size_t>(n));
    for (int64_t s = 0; s < n; ++s) by_key[size_t(kcount[size_t(key_of[size_t(s)])]++)] = s;
    std::vector<Src> v(static_cast<size_t>(n));
    for (int64_t r = 0; r < n; ++r) {
        const int64_t s = by_key[size_t(r)];
        const int32_t t = tile_of[size_t(s)];
        v[size_t(tcount[size_t(t)]++)] = Src{t, key_of[size_t(s)], ndot[s]};
    }
    // merge duplicate cells (nearest-grid-point projection sums them)
    Lists out;
    out.ptr.assign(size_t(g.nblocks) + 1, 0);
    std::vector<double> acc;
    std::vector<int32_t> tiles;
    for (size_t s = 0; s < v.size(); ++s) {
        if (!out.key.empty() && tiles.back() == v[s].tile && out.key.back() == v[s].key) {
            acc.back() += v[s].ndot;
        } else {
            tiles.push_back(v[s].tile);
            out.key.push_back(v[s].key);
            acc.push_back(v[s].ndot);
        }
    }
    const double vol = p.dx_cm * p.dx_cm * p.dx_cm;
    out.rate.resize(acc.size());
    for (size_t s = 0; s < acc.size(); ++s) out.rate[s] = float(acc[s] / vol);
    for (size_t s = 0; s < tiles.size(); ++s) out.ptr[size_t(tiles[s]) + 1] += 1;
    for (int b = 0; b < g.nblocks; ++b) out.ptr[size_t(b) + 1] += out.ptr[size_t(b)];
    return out;
}
}  // namespace

// Which tile set the next step uses: the LF forms take the 64 x TY_LF
// tiles when there are enough of them to fill the chip (four per compute
// unit), the 64 x TY ones on small grids; HLL takes the 64 x TY_HLL ones.
static int tile_set(const rt_ctx *c)
{
    if (c->p.flux == RT_FLUX_HLL) return 2;
    return c->geo[0].nblocks >= BIG_MIN_BLOCKS ? 0 : 1;
}

// Build tile set g's lists from the host copy of the sources.  New lists are
// allocated and filled first, so that a failure leaves the old ones intact.
static int build_lists(rt_ctx *c, int g)
{
    const int64_t n = int64_t(c->src_ndot.size());
    const Lists L = bin_sources(c, c->geo[g], n, c->src_ijk.data(), c->src_ndot.data());
    const size_t m = std::max<size_t>(L.key.size(), 1);
    int32_t *nkey = nullptr;
    float *nrate = nullptr;
    if (hipMalloc(&nkey, m * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&nrate, m * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        if (nkey) (void)hipFree(nkey);
        return RT_E_NOMEM;
    }
    if (!L.key.empty() &&
        (hipMemcpy(nkey, L.key.data(), L.key.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
             hipSuccess ||
         hipMemcpy(nrate, L.rate.data(), L.rate.size() * sizeof(float), hipMemcpyHostToDevice) !=
             hipSuccess)) {
        (void)hipFree(nkey);
        (void)hipFree(nrate);
        return RT_E_HIP;
    }
    // the stream may still read the old lists
    TileSet &t = c->geo[g];
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(t.d_src_ptr, L.ptr.data(), L.ptr.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(nkey);
        (void)hipFree(nrate);
        return RT_E_HIP;
    }
    if (t.d_src_key) (void)hipFree(t.d_src_key);
    if (t.d_src_rate) (void)hipFree(t.d_src_rate);
    t.d_src_key = nkey;
    t.d_src_rate = nrate;
    c->geo_ready[g] = true;
    return RT_OK;
}

int rtk::inject_host(rt_ctx *c, int64_t n, const int32_t *ijk, const double *ndot)
{
    const rt_params &p = c->p;
    double total = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const int32_t i = ijk[3 * s], j = ijk[3 * s + 1], k = ijk[3 * s + 2];
        const double q = ndot[s];
        if (i < 0 || i >= p.nx || j < 0 || j >= p.ny || k < 0 || k >= p.nz) return RT_E_ARG;
        if (!(q >= 0.0) || !isfinite(q)) return RT_E_ARG;
        total += q;
    }
    std::vector<int32_t> old_ijk;
    std::vector<double> old_ndot;
    old_ijk.swap(c->src_ijk);
    old_ndot.swap(c->src_ndot);
    c->src_ijk.assign(ijk, ijk + 3 * n);
    c->src_ndot.assign(ndot, ndot + n);
    // the set the next step uses now, the other one when first needed
    const int g = tile_set(c);
    const int rc = build_lists(c, g);
    if (rc != RT_OK) {
        c->src_ijk.swap(old_ijk);   // the old set stays, lists and all
        c->src_ndot.swap(old_ndot);
        return rc;
    }
    for (int o = 0; o < 3; ++o)
        if (o != g) c->geo_ready[o] = false;
    c->nsrc = int64_t(c->src_ndot.size());
    c->ndot_total = total;
    return RT_OK;
}

int rtk::check_clump(const rt_params &p)
{
    if (p.clump != 0 && p.clump != 1) return RT_E_ARG;
    if (p.clump == 1) {
        if (!(p.clump_cr_norm > 0.0) || !isfinite(p.clump_cr_norm)) return RT_E_ARG;
        if (!(p.clump_ci_norm > 0.0) || !isfinite(p.clump_ci_norm)) return RT_E_ARG;
        if (!(fabs(p.clump_cr_exp) <= 10.0) || !(fabs(p.clump_ci_exp) <= 10.0)) return RT_E_ARG;
    }
    return RT_OK;
}

ClumpLaw rtk::make_clump_law(const rt_params &p)
{
    ClumpLaw l{};
    l.on = p.clump;
    if (p.clump) {
        l.cr_exp = float(p.clump_cr_exp);
        l.cr_l2n = float(log2(p.clump_cr_norm));
        l.ci_exp = float(p.clump_ci_exp);
        l.ci_l2n = float(log2(p.clump_ci_norm));
    }
    return l;
}

ClumpLawD rtk::make_clump_law_d(const rt_params &p)
{
    ClumpLawD l{};
    l.on = p.clump;
    l.cr_norm = p.clump_cr_norm;
    l.cr_exp = p.clump_cr_exp;
    l.ci_norm = p.clump_ci_norm;
    l.ci_exp = p.clump_ci_exp;
    return l;
}

static void fill_args(const rt_ctx *c, double dt, int nsub, StepArgs &a)
{
    const rt_params &p = c->p;
    const int cur = c->cur, nxt = 1 - c->cur;
    a.N = c->f.N[cur];
    a.Fx = c->f.Fx[cur];
    a.Fy = c->f.Fy[cur];
    a.Fz = c->f.Fz[cur];
    a.No = c->f.N[nxt];
    a.Fxo = c->f.Fx[nxt];
    a.Fyo = c->f.Fy[nxt];
    a.Fzo = c->f.Fz[nxt];
    a.xHI = c->f.xHI;
    a.T = c->f.T;
    a.nH = c->f.nH;
    const int gi = tile_set(c);
    const TileSet &g = c->geo[gi];
    a.big = gi == 0 ? 1 : 0;
    a.src_ptr = g.d_src_ptr;
    a.src_key = g.d_src_key;
    a.src_rate = g.d_src_rate;
    a.partials = c->d_part;
    a.sink = c->d_sink;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.plane = uint32_t(p.nx) * uint32_t(p.ny);
    a.ntx = c->ntx;
    a.nty = g.nty;
    a.nzc = g.nzc;
    a.zc = g.zc;
    a.nblocks = g.nblocks;
    for (int f = 0; f < 6; ++f) a.bc[f] = p.bc[f];
    a.chem = p.chem;
    a.mixed = p.prec == RT_PREC_MIXED;
    a.adaptive = p.sub == RT_SUB_ADAPTIVE;
    a.nsub = nsub;
    a.cl = make_clump_law(p);
    a.cld = make_clump_law_d(p);
    a.any_outflow = 0;
    for (int f = 0; f < 6; ++f) a.any_outflow |= p.bc[f] == RT_BC_OUTFLOW ? 1 : 0;
    const double c_ = p.c_cms;
    const double eheat = (p.sigma_e * p.egamma_eV / p.sigma_n - E_ION_EV) * EV;
    const double T_h = eheat / (1.5 * KB);
    a.c = float(c_);
    a.inv_c = float(1.0 / c_);
    a.half_c = float(0.5 * c_);
    a.half_c2 = float(0.5 * c_ * c_);
    a.k1 = float(dt / p.dx_cm);
    a.dt = float(dt);
    a.csig = float(c_ * p.sigma_n);
    a.T_h = float(T_h);
    a.inv15kB = float(1.0 / (1.5 * KB));
    a.T_floor = float(p.T_floor);
    a.sub_eps = float(p.sub_eps);
    a.xhi_thr = float(p.xhi_fp64_thr);
    a.dt_d = dt;
    a.csig_d = c_ * p.sigma_n;
    a.T_h_d = T_h;
    a.T_floor_d = p.T_floor;
    a.sub_eps_d = p.sub_eps;
    a.inv15kB_d = 1.0 / (1.5 * KB);
    a.vol = p.dx_cm * p.dx_cm * p.dx_cm;
    a.esc_scale = dt * p.dx_cm * p.dx_cm;
    a.hll = p.flux == RT_FLUX_HLL ? 1 : 0;
    // stiff cells leave the step for the dense deferred kernel in the
    // adaptive and learned forms
    a.defer_stiff = (p.chem != RT_CHEM_OFF && (c->surr || p.sub == RT_SUB_ADAPTIVE)) ? 1 : 0;
    a.defer = (p.chem != RT_CHEM_OFF && (p.prec == RT_PREC_MIXED || a.defer_stiff)) ? 1 : 0;
    a.count_hist = (p.sub == RT_SUB_ADAPTIVE || c->surr) ? 1 : 0;
    a.fp64_mask = c->d_mask;
    a.group_mask = c->d_gmask;
    a.c_d = p.c_cms;
    a.surr = c->surr ? 1 : 0;
    a.surr_pk = c->d_surr_pk;
    a.surr_bias = c->d_surr_bias;
    for (int k = 0; k < SURR_NNORM; ++k) a.surr_norm[k] = c->surr_norm[k];
    a.surr_tol = c->surr_tol;
    a.log10_dt = float(log10(dt));
    a.expand = c->hubble > 0.0 ? 1 : 0;
    a.dil3 = float(exp(-3.0 * c->hubble * dt));
    a.dil2 = float(exp(-2.0 * c->hubble * dt));
    a.one_m_dil3 = float(-expm1(-3.0 * c->hubble * dt));
}

extern "C" int rt_set_expansion(rt_ctx *c, double hubble)
{
    if (!c) return RT_E_STATE;
    if (!(hubble >= 0.0) || !isfinite(hubble)) return RT_E_ARG;
    c->hubble = hubble;
    return RT_OK;
}

extern "C" int rt_step(rt_ctx *c, double dt, int32_t nsub)
{
    if (!c) return RT_E_STATE;
    if (!(dt > 0.0) || !isfinite(dt)) return RT_E_ARG;
    if (nsub < 1 || nsub > MAX_NSUB) return RT_E_ARG;
    const double dtmax = c->p.dx_cm / (3.0 * c->p.c_cms);
    if (dt > dtmax * (1.0 + 1e-12)) return RT_E_CFL;

    if (!c->geo_ready[tile_set(c)]) {
        const int rc = build_lists(c, tile_set(c));
        if (rc != RT_OK) return rc;
    }
    StepArgs a;
    fill_args(c, dt, nsub, a);
    const int rows = a.nblocks + defer_rows(a, c->nb2);
    if (rows > c->npart) return RT_E_STATE;   // the partials would not fit
    if (a.defer && (!c->d_mask || !c->d_gmask || !c->d_goff || !c->d_cells)) return RT_E_STATE;
    if (a.surr && !c->d_mask2) return RT_E_STATE;
    Ev *e = nullptr;
    if (c->prof) {
        if (c->ev_used == c->ev.size()) {
            Ev n;
            if (hipEventCreate(&n.a) != hipSuccess) return RT_E_HIP;
            if (hipEventCreate(&n.b) != hipSuccess) return RT_E_HIP;
            c->ev.push_back(n);
        }
        e = &c->ev[c->ev_used++];
        if (hipEventRecord(e->a, c->stream) != hipSuccess) return RT_E_HIP;
    }
    if (launch_step(a, c->stream) != hipSuccess) return RT_E_HIP;
    if (a.defer &&
        launch_defer_chem(a, c->nwords, c->nb2, c->d_goff, c->d_cells, c->d_mask2, c->stream) !=
            hipSuccess)
        return RT_E_HIP;
    if (e && hipEventRecord(e->b, c->stream) != hipSuccess) return RT_E_HIP;
    const double tau_coef = c->p.c_cms * SIGMA_T * dt / double(c->ncell);
    if (launch_finalize(c->d_part, rows, c->d_fin, c->d_acc, 0, tau_coef, c->nh_sum,
                        c->stream, a.defer ? c->d_gmask : nullptr, a.defer ? c->gwords : 0) !=
        hipSuccess)
        return RT_E_HIP;
    c->cur = 1 - c->cur;
    c->t += dt;
    c->emitted += dt * c->ndot_total;
    c->steps += 1;
    if (!a.count_hist && c->p.chem != RT_CHEM_OFF) {
        int b = 0;
        while (b < 7 && (2 << b) <= nsub) ++b;
        c->hist_host[b] += int64_t(c->ncell);
    }
    return RT_OK;
}

extern "C" int rt_set_surrogate(rt_ctx *c, const float *theta, const float *norm,
                                double residual_tol)
{
    if (!c) return RT_E_STATE;
    if (!theta) {
        c->surr = false;
        return RT_OK;
    }
    if (!norm || !(residual_tol > 0.0) || !isfinite(residual_tol)) return RT_E_ARG;
    // the stiffness test that selects the network's cells uses sub_eps
    if (!(c->p.sub_eps >= 0.0 && c->p.sub_eps <= 1.0)) return RT_E_ARG;
    for (int k = 0; k < SURR_NNORM; ++k)
        if (!isfinite(norm[k])) return RT_E_ARG;
    for (int k = 0; k < 7; ++k)
        if (!(norm[5 + k < 10 ? 5 + k : 12 + (k - 5)] > 0.0f)) return RT_E_ARG;
    for (int k = 0; k < 5; ++k)
        if (!(norm[14 + k] <= norm[19 + k])) return RT_E_ARG;
    if (!c->d_surr_pk) {
        if (hipMalloc(&c->d_surr_pk, size_t(PK_ALL) * 8 * sizeof(__bf16)) != hipSuccess ||
            hipMalloc(&c->d_surr_bias, SURR_NBIAS * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return RT_E_NOMEM;
        }
    }
    {
        const int rc = alloc_masks(c);
        if (rc != RT_OK) return rc;
    }
    if (!c->d_mask2 && hipMalloc(&c->d_mask2, c->nwords * sizeof(uint64_t)) != hipSuccess) {
        (void)hipGetLastError();
        return RT_E_NOMEM;
    }
    const int offs[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
    const int lens[4] = {MLP_NH, MLP_NH, MLP_NH, MLP_NOUT};
    int at = 0;
    if (launch_mlp_pack(theta, c->d_surr_pk, c->stream) != hipSuccess) return RT_E_HIP;
    for (int l = 0; l < 4; ++l) {
        if (hipMemcpyAsync(c->d_surr_bias + at, theta + offs[l], lens[l] * sizeof(float),
                           hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return RT_E_HIP;
        at += lens[l];
    }
    for (int k = 0; k < SURR_NNORM; ++k) c->surr_norm[k] = norm[k];
    c->surr_tol = float(residual_tol);
    c->surr = true;
    return RT_OK;
}

extern "C" int rt_reduce(rt_ctx *c, rt_reductions *out)
{
    if (!c) return RT_E_STATE;
    if (!out) return RT_E_ARG;
    double acc[ACC_SIZE];
    if (hipMemcpyAsync(acc, c->d_acc, sizeof(acc), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return RT_E_HIP;
    const rt_params &p = c->p;
    const double vol = p.dx_cm * p.dx_cm * p.dx_cm;
    const double ncell = double(c->ncell);
    memset(out, 0, sizeof(*out));
    out->t = c->t;
    out->xhi_vol = acc[ACC_CUR + R_XHI] / ncell;
    out->xhi_mass = acc[ACC_CUR + R_NHXHI] / c->nh_sum;
    out->gamma_vol = p.c_cms * p.sigma_n * acc[ACC_CUR + R_N] / ncell;
    out->photons_initial = c->photons_initial;
    out->photons_emitted = c->emitted;
    out->photons_stored = acc[ACC_CUR + R_N] * vol;
    out->photons_absorbed = acc[ACC_CUM + R_ABS];
    out->photons_escaped = acc[ACC_CUM + R_ESC];
    out->photons_floor = acc[ACC_CUM + R_FLOOR];
    out->photons_diluted = acc[ACC_CUM + R_DILUTE];
    out->steps = c->steps;
    out->n_nonfinite = int64_t(acc[ACC_CUM + R_NONFINITE]);
    out->n_fp64 = int64_t(acc[ACC_CUM + R_FP64]);
    out->n_fallback = int64_t(acc[ACC_CUM + R_FALLBACK]);
    for (int b = 0; b < 8; ++b)
        out->subcycle_hist[b] = c->hist_host[b] + int64_t(acc[ACC_CUM + R_HIST0 + b]);
    out->tau_e = acc[ACC_CUM + ACC_TAU];
    out->n_learned = int64_t(acc[ACC_CUM + R_LEARNED]);
    out->n_fallback_range = int64_t(acc[ACC_CUM + R_RANGE]);
    return out->n_nonfinite > 0 ? RT_E_NONFINITE : RT_OK;
}

extern "C" int rt_equilibrium_xhi(const rt_params *p, int32_t model, double gamma0,
                                  double n_star, int64_t n, const double *nH, const double *T,
                                  double *xhi, void *hip_stream)
{
    if (!p || check_clump(*p) != RT_OK) return RT_E_ARG;
    if (model < RT_JMODEL_UNIFORM || model > RT_JMODEL_EXP4) return RT_E_ARG;
    if (!(gamma0 >= 0.0) || !isfinite(gamma0)) return RT_E_ARG;
    if (model != RT_JMODEL_UNIFORM && (!(n_star > 0.0) || !isfinite(n_star))) return RT_E_ARG;
    if (n < 0 || n > (int64_t(1) << 31) - 1) return RT_E_ARG;
    if (n == 0) return RT_OK;
    if (!nH || !T || !xhi) return RT_E_ARG;
    const hipError_t e = launch_equilibrium(n, nH, T, xhi, model, gamma0, n_star, *p,
                                            static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? RT_OK : RT_E_HIP;
}

extern "C" int rt_histogram(rt_ctx *c, int32_t quantity, int32_t nbx, double lox, double hix,
                            int32_t nby, double loy, double hiy, int64_t *counts,
                            double *sum_q)
{
    if (!c) return RT_E_STATE;
    if (quantity != RT_HQ_XHI && quantity != RT_HQ_GAMMA) return RT_E_ARG;
    if (nbx < 1 || nbx > 256 || nby < 1 || nby > 256 || nbx * nby > RT_HIST_MAX_BINS)
        return RT_E_ARG;
    for (double v : {lox, hix, loy, hiy})
        if (!(fabs(v) <= 300.0)) return RT_E_ARG;
    if (!(lox < hix) || !(loy < hiy)) return RT_E_ARG;
    if (!counts || !sum_q) return RT_E_ARG;
    // edges e_k = 10^(lo + k w), w = (hi - lo) / nb, in FP64
    double h_edges[2 * 257];
    const double wx = (hix - lox) / nbx, wy = (hiy - loy) / nby;
    for (int k = 0; k <= nbx; ++k) h_edges[k] = pow(10.0, lox + k * wx);
    for (int k = 0; k <= nby; ++k) h_edges[nbx + 1 + k] = pow(10.0, loy + k * wy);
    double *d_sum = c->d_hsum, *d_edges = c->d_hsum + 256;
    const float *q = quantity == RT_HQ_XHI ? c->f.xHI : c->f.N[c->cur];
    std::vector<unsigned long long> hc(size_t(nbx) * nby);
    if (hipMemcpyAsync(d_edges, h_edges, size_t(nbx + nby + 2) * sizeof(double),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_hcount, 0, hc.size() * sizeof(unsigned long long), c->stream) !=
            hipSuccess ||
        hipMemsetAsync(c->d_hlimb, 0, hist_limb_count(nbx) * sizeof(unsigned long long),
                       c->stream) != hipSuccess ||
        launch_hist(c->f.nH, q, quantity == RT_HQ_GAMMA, c->p.c_cms * c->p.sigma_n, c->ncell,
                    nbx, nby, d_edges, float(lox), float(1.0 / wx), float(loy),
                    float(1.0 / wy), c->d_hcount, c->d_hlimb, d_sum, c->stream) != hipSuccess ||
        hipMemcpyAsync(hc.data(), c->d_hcount, hc.size() * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(sum_q, d_sum, size_t(nbx) * sizeof(double), hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return RT_E_HIP;
    for (size_t i = 0; i < hc.size(); ++i) counts[i] = int64_t(hc[i]);
    return RT_OK;
}

extern "C" int rt_gamma_plateau(rt_ctx *c, double nH_max, double *gamma0, int64_t *ncells)
{
    if (!c) return RT_E_STATE;
    if (!gamma0 || !(nH_max > 0.0) || !isfinite(nH_max)) return RT_E_ARG;
    double h[2] = {0.0, 0.0};
    if (launch_plateau(c->f.nH, c->f.N[c->cur], c->ncell, nH_max, c->p.c_cms * c->p.sigma_n,
                       c->d_part, c->d_fin, c->stream) != hipSuccess ||
        hipMemcpyAsync(h, c->d_fin, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return RT_E_HIP;
    if (ncells) *ncells = int64_t(h[1]);
    if (!(h[1] > 0.0)) return RT_E_ARG;
    *gamma0 = h[0] / h[1];
    return RT_OK;
}

extern "C" int rt_state(rt_ctx *c, int32_t field, void *dst, int32_t dst_on_device)
{
    if (!c) return RT_E_STATE;
    if (!dst) return RT_E_ARG;
    const void *src = nullptr;
    switch (field) {
    case RT_FIELD_N: src = c->f.N[c->cur]; break;
    case RT_FIELD_FX: src = c->f.Fx[c->cur]; break;
    case RT_FIELD_FY: src = c->f.Fy[c->cur]; break;
    case RT_FIELD_FZ: src = c->f.Fz[c->cur]; break;
    case RT_FIELD_XHI: src = c->f.xHI; break;
    case RT_FIELD_T: src = c->f.T; break;
    case RT_FIELD_NH: src = c->f.nH; break;
    default: return RT_E_ARG;
    }
    const size_t bytes = size_t(c->ncell) * sizeof(float);
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (hipMemcpyAsync(dst, src, bytes, kind, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return RT_E_HIP;
    return RT_OK;
}

extern "C" int rt_current(rt_ctx *c, int32_t *index)
{
    if (!c) return RT_E_STATE;
    if (!index) return RT_E_ARG;
    *index = c->cur;
    return RT_OK;
}

extern "C" int rt_profile(rt_ctx *c, int32_t enable)
{
    if (!c) return RT_E_STATE;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return RT_E_HIP;
    c->prof = enable != 0;
    c->ev_used = 0;
    return RT_OK;
}

extern "C" int rt_profile_read(rt_ctx *c, double *ms_total, int64_t *launches)
{
    if (!c) return RT_E_STATE;
    if (!ms_total || !launches) return RT_E_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return RT_E_HIP;
    double tot = 0.0;
    for (size_t i = 0; i < c->ev_used; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev[i].a, c->ev[i].b) != hipSuccess) return RT_E_HIP;
        tot += ms;
    }
    *ms_total = tot;
    *launches = int64_t(c->ev_used);
    return RT_OK;
}

extern "C" int rt_destroy(rt_ctx *c)
{
    if (!c) return RT_E_STATE;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
    return RT_OK;
}
