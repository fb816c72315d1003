// rt_step.hip -- gfx950 kernels of one explicit M1 radiative-transfer step
// fused with the per-cell hydrogen chemistry (Aubert & Teyssier 2010,
// Sec. 2.2 and Appendix A).
//
// Fused step kernel, one pass over HBM per step:
//   * a block owns a 64 x 8 (x, y) tile and marches ZC planes along z; each
//     of its 8 wavefronts holds one coalesced 64-cell x-row (the paper's
//     "horizontal" thread layout, Appendix A);
//   * plane z of (N, F) and its M1 pressure tensor sit in LDS with a one-cell
//     x/y halo whose boundary images (periodic wrap, outflow copy, reflection)
//     are produced by the loader, so the grid carries no ghost layers;
//   * planes z-1 and z+1 of the thread's own column stay in registers;
//   * the unsplit Lax-Friedrichs (or HLL) update, the point sources, the
//     positivity guards, the chemistry Phi and the FP64 global sums all
//     happen on values already in registers; each cell is read and written
//     exactly once;
//   * cells whose chemistry is expensive or needs FP64 -- the stiff cells
//     of the adaptive and learned forms, the ionised cells of the mixed
//     form -- are marked in a bit mask and left to a second kernel that
//     gathers them into dense wavefronts (the network runs there on the
//     matrix cores), so that the bandwidth-bound sweep never waits on
//     divergent sub-cycles;
//   * blocks are renumbered so that each XCD (blockIdx mod 8) receives a
//     contiguous run of neighbouring tiles and shares their halo rows in its
//     own L2.
#include <math.h>

#include <algorithm>

#include "mlp_device.h"

#ifndef RT_M1_NT_STORES
#define RT_M1_NT_STORES 1
#endif

namespace rtk {

// ------------------------------------------------------ boundary mapping
struct Map1 {
    int idx;
    float sign;  // -1 where the image reflects the normal flux
};

__device__ __forceinline__ Map1 map_coord(int g, int n, int bc_lo, int bc_hi)
{
    Map1 m{g, 1.0f};
    if (g < 0) {
        if (bc_lo == RT_BC_PERIODIC) {
            int r = g % n;
            m.idx = r < 0 ? r + n : r;
        } else {
            m.idx = 0;
            if (bc_lo == RT_BC_REFLECT) m.sign = -1.0f;
        }
    } else if (g >= n) {
        if (bc_hi == RT_BC_PERIODIC) {
            m.idx = g % n;
        } else {
            m.idx = n - 1;
            if (bc_hi == RT_BC_REFLECT) m.sign = -1.0f;
        }
    }
    return m;
}

// Results are not re-read by this kernel: stream them past the caches so
// that L2 keeps the halo rows shared by neighbouring tiles.
__device__ __forceinline__ void store_out(float *p, float v)
{
#if RT_M1_NT_STORES
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

struct Cell4 {
    float N, Fx, Fy, Fz;
};

// Prefetches stay raw: applying a reflection sign at load time would make
// the kernel wait for the load right where it is issued.
__device__ __forceinline__ Cell4 load_raw(const StepArgs &A, uint32_t i)
{
    Cell4 c;
    c.N = A.N[i];
    c.Fx = A.Fx[i];
    c.Fy = A.Fy[i];
    c.Fz = A.Fz[i];
    return c;
}

__device__ __forceinline__ Cell4 signed4(const Cell4 &r, float sx, float sy, float sz)
{
    return Cell4{r.N, sx * r.Fx, sy * r.Fy, sz * r.Fz};
}

__device__ __forceinline__ Cell4 load4(const StepArgs &A, uint32_t i, float sx, float sy,
                                       float sz)
{
    Cell4 c;
    c.N = A.N[i];
    c.Fx = sx * A.Fx[i];
    c.Fy = sy * A.Fy[i];
    c.Fz = sz * A.Fz[i];
    return c;
}

// ------------------------------------------------------ fused step kernel
// One block per CU.  On large grids the LF forms take 64 x 16 tiles (BIG):
// 1024 threads at up to 128 VGPRs, four wavefronts per SIMD; on small grids
// 64 x 8 tiles: 512 threads at up to 256 VGPRs.  The HLL form takes 64 x 12
// tiles: 768 threads at up to 168 VGPRs, three wavefronts per SIMD (measured
// 14.63 against 15.59 ms per 1024^3 step on 64 x 8 tiles at 187 VGPRs, 2.02
// against 2.33 ms at 512^3; the small LF form was 14% slower at 128^3 on
// 64 x 12 tiles, which leave fewer blocks).
#ifndef RT_M1_MINW
#define RT_M1_MINW 2
#endif
#ifndef RT_M1_MINW_LF
#define RT_M1_MINW_LF 4
#endif
#ifndef RT_M1_MINW_HLL
#define RT_M1_MINW_HLL 3
#endif

template <bool HLL, bool BIG>
__global__ __launch_bounds__(BIG ? NTHREADS_LF : (HLL ? NTHREADS_HLL : NTHREADS),
                             BIG ? RT_M1_MINW_LF : (HLL ? RT_M1_MINW_HLL : RT_M1_MINW))
void m1_step_kernel(StepArgs A)
{
    static_assert(!BIG || !HLL, "64 x 16 tiles: LF forms only");
    constexpr int KTY = BIG ? TY_LF : (HLL ? TY_HLL : TY);   // tile rows of this form
    constexpr int KNT = TX * KTY;           // its threads per block
    constexpr int SW = TX + 2;
    // Plane z's tile and halo, double-buffered by the parity of z: a plane
    // writes one buffer while slower wavefronts may still read the other,
    // so one barrier per plane suffices (everyone has finished reading a
    // buffer before anyone passes the barrier of the plane after it).
    __shared__ float sN[2][KTY + 2][SW], sFx[2][KTY + 2][SW], sFy[2][KTY + 2][SW];
    __shared__ float sFz[2][KTY + 2][SW];
    __shared__ float sPxx[2][KTY + 2][SW], sPyy[2][KTY + 2][SW], sPxy[2][KTY + 2][SW];
    __shared__ float sPxz[2][KTY + 2][SW], sPyz[2][KTY + 2][SW];
    // HLL: x and y signal speeds of the tile and its halo
    constexpr int HY = HLL ? KTY + 2 : 1, HX = HLL ? SW : 1;
    __shared__ float sLxm[2][HY][HX], sLxp[2][HY][HX], sLym[2][HY][HX], sLyp[2][HY][HX];
    __shared__ double sred[KNT / 64][NRED];

    const int tid = threadIdx.x;
    const int lx = tid & (TX - 1), ly = tid / TX;

    // XCD-aware band order.  blockIdx mod 8 selects the XCD; every run of
    // 256 blocks (one per compute unit, dispatched together) covers 256
    // consecutive tiles (x fastest), 32 of them per XCD, so that the tiles
    // resident at any time form one contiguous band of whole tile rows that
    // marches z side by side: the x- and y-halo cells a tile reads were
    // fetched moments earlier by its neighbours, into the same XCD's L2 (or,
    // across XCDs, the memory-side cache).  Measured at 1024^3: 12.21 ms per
    // step against 12.74 for contiguous per-XCD ranges, whose neighbouring
    // tile rows ran 32 planes apart; a band order taking z chunks before y
    // was slower (13.8 ms).  The blocks of the last, partial run keep their
    // index.
    const int b = blockIdx.x, nb = A.nblocks;
    const int xcd = b & 7, slot = b >> 3;
    const int tile = b < (nb & ~255) ? (slot >> 5) * 256 + xcd * 32 + (slot & 31) : b;
    const int itx = tile % A.ntx;
    const int rest = tile / A.ntx;
    const int ity = rest % A.nty;
    const int izc = rest / A.nty;
    const int tile_id = tile;   // source-list index
    const int x0 = itx * TX, y0 = ity * KTY;
    const int z0 = izc * A.zc;
    const int z1 = min(z0 + A.zc, A.nz);
    const int gx = x0 + lx, gy = y0 + ly;
    const bool active = gx < A.nx && gy < A.ny;
    const uint32_t plane = A.plane;

    // own column (boundary image for slots outside the grid)
    const Map1 mx = map_coord(gx, A.nx, A.bc[0], A.bc[1]);
    const Map1 my = map_coord(gy, A.ny, A.bc[2], A.bc[3]);
    const uint32_t col = uint32_t(my.idx) * uint32_t(A.nx) + uint32_t(mx.idx);

    // halo slot of this thread: rows y0-1 and y0+KTY, columns x0-1 and x0+TX
    int hsx = 0, hsy = 0;
    const bool has_halo = tid < 2 * TX + 2 * KTY;
    if (tid < TX) {
        hsy = 0;
        hsx = tid + 1;
    } else if (tid < 2 * TX) {
        hsy = KTY + 1;
        hsx = tid - TX + 1;
    } else if (tid < 2 * TX + KTY) {
        hsx = 0;
        hsy = tid - 2 * TX + 1;
    } else {
        hsx = TX + 1;
        hsy = tid - 2 * TX - KTY + 1;
    }
    const Map1 hx = map_coord(x0 + hsx - 1, A.nx, A.bc[0], A.bc[1]);
    const Map1 hy = map_coord(y0 + hsy - 1, A.ny, A.bc[2], A.bc[3]);
    const uint32_t hcol = uint32_t(hy.idx) * uint32_t(A.nx) + uint32_t(hx.idx);

    // Sources of this tile, sorted by plane, staged in LDS (refilled when
    // exhausted): the walk then waits on LDS only and never drains the
    // prefetched global loads in flight.
    __shared__ int s_skey[SRC_LDS];
    __shared__ float s_srate[SRC_LDS];
    int sp = A.src_ptr[tile_id];
    const int sp_end = A.src_ptr[tile_id + 1];
    int buf_base = sp;
    int buf_n = min(SRC_LDS, sp_end - sp);
    for (int i = tid; i < buf_n; i += KNT) {
        s_skey[i] = A.src_key[buf_base + i];
        s_srate[i] = A.src_rate[buf_base + i];
    }

    // FP64 sums.  The four that change every plane are accumulated per
    // thread (a per-plane wavefront reduction was measured to cost ~25% of
    // the step); escaped and floor photons, which are zero almost
    // everywhere, are reduced across the wavefront only on planes where
    // they occur and kept per wavefront in LDS.
    __shared__ double s_acc[KNT / 64][8];
    const int wave = tid >> 6;
    if (lx < 8) s_acc[wave][lx] = 0.0;
    double acc_xhi = 0.0, acc_nhxhi = 0.0, acc_N = 0.0, acc_abs = 0.0;
    int n_bad = 0;
    __shared__ int shist[8];
    if (tid < 8) shist[tid] = 0;

    const ChemK<float> Kf{A.dt,      A.dt / float(A.nsub), A.csig,   A.T_h,
                          A.T_floor, A.sub_eps,            A.inv15kB};

    // prologue: plane z0-1 (boundary image if outside), plane z0, plane z0+1
    const Map1 mzm = map_coord(z0 - 1, A.nz, A.bc[4], A.bc[5]);
    Cell4 prv = load4(A, col + uint32_t(mzm.idx) * plane, mx.sign, my.sign, mzm.sign);
    // the HLL form carries c^2 P (the flux of F along each axis) and takes
    // the pressure and the signal speeds of a cell in one pass
    const float pscale = HLL ? 2.0f * A.half_c2 : 1.0f;
    auto press_speeds = [&](const Cell4 &u, Press &P, Speeds &L) {
        if constexpr (HLL) {
            SpeedPrep sp;
            closure_and_prep(u.N, u.Fx, u.Fy, u.Fz, A.inv_c, A.c_d, pscale, P, sp);
            L = m1_axes(sp);
        } else {
            P = closure(u.N, u.Fx, u.Fy, u.Fz, A.inv_c);
        }
    };
    Press pprv, pcur;
    Speeds lprv{}, lcur{};
    press_speeds(prv, pprv, lprv);
    Cell4 cur = load4(A, col + uint32_t(z0) * plane, mx.sign, my.sign, 1.0f);
    press_speeds(cur, pcur, lcur);
    // HLL signal speeds travel with the z window like the pressure tensors.
    // The z face below plane z is the face above plane z-1: its HLL weights
    // are carried from one plane to the next.
    HllW wz_prev{};
    if constexpr (HLL) wz_prev = hll_weights(lprv.zm, lprv.zp, lcur.zm, lcur.zp, A.c);
    // Prefetched planes live in two register sets that swap roles every
    // plane: the loop below is unrolled by two so that a value loaded for
    // the next plane is never copied, and its load stays in flight across
    // the plane boundary instead of being waited for at the end of an
    // iteration.  Set k holds the planes z with (z - z0) % 2 == k.  (A
    // two-plane prefetch distance was measured to gain nothing.)
    const uint32_t hsrc = has_halo ? hcol : col;
    const float hsx_sign = has_halo ? hx.sign : 1.0f, hsy_sign = has_halo ? hy.sign : 1.0f;
    auto load_ch = [&](float3 &c, int zz) {
        const uint32_t i = col + uint32_t(zz) * plane;
        // read once per step by this thread alone: non-temporal loads keep
        // them from displacing the N, F lines that neighbouring tiles read
        // as halo (measured 1.5% faster; N, F loaded so were 3-20% slower)
        c.x = __builtin_nontemporal_load(&A.xHI[i]);
        c.y = __builtin_nontemporal_load(&A.T[i]);
        c.z = __builtin_nontemporal_load(&A.nH[i]);
    };
    const Cell4 zero4{0.f, 0.f, 0.f, 0.f};
    const float3 zero3 = make_float3(0.f, 0.f, 0.f);
    Cell4 nx0 = zero4, nx1 = zero4;
    Cell4 ha0 = zero4, ha1 = zero4;
    float3 ch0 = zero3, ch1 = zero3;
    nx1 = load_raw(A, col + uint32_t(map_coord(z0 + 1, A.nz, A.bc[4], A.bc[5]).idx) * plane);
    ha0 = load_raw(A, hsrc + uint32_t(z0) * plane);
    load_ch(ch0, z0);

    // One plane z.  nxt: plane z+1 of the own column (loaded earlier);
    // nx_ld receives plane z+2.  hal: this thread's halo cell of plane z;
    // hal_ld receives plane z+1's.  ch: xHI, T, nH of plane z; ch_ld
    // receives plane z+1's.
    uint64_t mword = 0;   // A.defer: this lane's plane (z0 + lane) of deferred cells
    auto plane_step = [&](const int z, const Cell4 &nxt_raw, Cell4 &nx_ld, const Cell4 &hal_raw,
                          Cell4 &hal_ld, const float3 &ch, float3 &ch_ld, const int bi) {
        const float c_xh = ch.x, c_nh = ch.z;
        float c_T = ch.y;
        // Prefetch (unconditionally, so that every lane of every plane issues
        // the same loads and the compiler's count of outstanding memory
        // operations stays exact: non-halo lanes re-load their own cell, the
        // chunk's last plane loads a valid neighbour that is not used).
        {
            const Map1 mzq = map_coord(z + 2, A.nz, A.bc[4], A.bc[5]);
            const int zh = z + 1 < z1 ? z + 1 : z;
            nx_ld = load_raw(A, col + uint32_t(mzq.idx) * plane);
            hal_ld = load_raw(A, hsrc + uint32_t(zh) * plane);
            load_ch(ch_ld, zh);
        }

        // boundary-image signs of the prefetched planes, applied on use
        const Cell4 nxt = signed4(nxt_raw, mx.sign, my.sign,
                                  map_coord(z + 1, A.nz, A.bc[4], A.bc[5]).sign);
        const Cell4 hal = signed4(hal_raw, hsx_sign, hsy_sign, 1.0f);

        // plane z into LDS: own cell and its halo
        {
            const int sy = ly + 1, sx = lx + 1;
            sN[bi][sy][sx] = cur.N;
            sFx[bi][sy][sx] = cur.Fx;
            sFy[bi][sy][sx] = cur.Fy;
            sFz[bi][sy][sx] = cur.Fz;
            sPxx[bi][sy][sx] = pcur.xx;
            sPyy[bi][sy][sx] = pcur.yy;
            sPxy[bi][sy][sx] = pcur.xy;
            sPxz[bi][sy][sx] = pcur.xz;
            sPyz[bi][sy][sx] = pcur.yz;
            if constexpr (HLL) {
                sLxm[bi][sy][sx] = lcur.xm;
                sLxp[bi][sy][sx] = lcur.xp;
                sLym[bi][sy][sx] = lcur.ym;
                sLyp[bi][sy][sx] = lcur.yp;
            }
        }
        if (has_halo) {
            Press ph;
            SpeedPrep ph2;
            if constexpr (HLL)
                closure_and_prep(hal.N, hal.Fx, hal.Fy, hal.Fz, A.inv_c, A.c_d, pscale, ph, ph2);
            else
                ph = closure(hal.N, hal.Fx, hal.Fy, hal.Fz, A.inv_c);
            sN[bi][hsy][hsx] = hal.N;
            sFx[bi][hsy][hsx] = hal.Fx;
            sFy[bi][hsy][hsx] = hal.Fy;
            sFz[bi][hsy][hsx] = hal.Fz;
            sPxx[bi][hsy][hsx] = ph.xx;
            sPyy[bi][hsy][hsx] = ph.yy;
            sPxy[bi][hsy][hsx] = ph.xy;
            sPxz[bi][hsy][hsx] = ph.xz;
            sPyz[bi][hsy][hsx] = ph.yz;
            if constexpr (HLL) {
                // a halo row is read for its y speeds only, a halo column for
                // its x speeds (whole wavefronts take the same branch)
                float lm, lp;
                if (tid < 2 * TX) {
                    m1_axis(ph2, ph2.uy, ph2.y2, ph2.x2 + ph2.z2, lm, lp);
                    sLym[bi][hsy][hsx] = lm;
                    sLyp[bi][hsy][hsx] = lp;
                } else {
                    m1_axis(ph2, ph2.ux, ph2.x2, ph2.y2 + ph2.z2, lm, lp);
                    sLxm[bi][hsy][hsx] = lm;
                    sLxp[bi][hsy][hsx] = lp;
                }
            }
        }
        __syncthreads();

        Press pnxt;
        Speeds lnxt{};
        press_speeds(nxt, pnxt, lnxt);
        const int sy = ly + 1, sx = lx + 1;
        // neighbours: x-1 (L), x+1 (R), y-1 (D), y+1 (U), z-1 (prv), z+1 (nxt)
        const float NL = sN[bi][sy][sx - 1], NR = sN[bi][sy][sx + 1];
        const float ND = sN[bi][sy - 1][sx], NU = sN[bi][sy + 1][sx];
        const float FxL = sFx[bi][sy][sx - 1], FxR = sFx[bi][sy][sx + 1];
        const float FxD = sFx[bi][sy - 1][sx], FxU = sFx[bi][sy + 1][sx];
        const float FyL = sFy[bi][sy][sx - 1], FyR = sFy[bi][sy][sx + 1];
        const float FyD = sFy[bi][sy - 1][sx], FyU = sFy[bi][sy + 1][sx];
        const float FzL = sFz[bi][sy][sx - 1], FzR = sFz[bi][sy][sx + 1];
        const float FzD = sFz[bi][sy - 1][sx], FzU = sFz[bi][sy + 1][sx];
        const float PxxL = sPxx[bi][sy][sx - 1], PxxR = sPxx[bi][sy][sx + 1];
        const float PxyL = sPxy[bi][sy][sx - 1], PxyR = sPxy[bi][sy][sx + 1];
        const float PxzL = sPxz[bi][sy][sx - 1], PxzR = sPxz[bi][sy][sx + 1];
        const float PxyD = sPxy[bi][sy - 1][sx], PxyU = sPxy[bi][sy + 1][sx];
        const float PyyD = sPyy[bi][sy - 1][sx], PyyU = sPyy[bi][sy + 1][sx];
        const float PyzD = sPyz[bi][sy - 1][sx], PyzU = sPyz[bi][sy + 1][sx];
        float lxmL = 0.f, lxpL = 0.f, lxmR = 0.f, lxpR = 0.f;
        float lymD = 0.f, lypD = 0.f, lymU = 0.f, lypU = 0.f;
        if constexpr (HLL) {
            lxmL = sLxm[bi][sy][sx - 1];
            lxpL = sLxp[bi][sy][sx - 1];
            lxmR = sLxm[bi][sy][sx + 1];
            lxpR = sLxp[bi][sy][sx + 1];
            lymD = sLym[bi][sy - 1][sx];
            lypD = sLyp[bi][sy - 1][sx];
            lymU = sLym[bi][sy + 1][sx];
            lypU = sLyp[bi][sy + 1][sx];
        }

        float dN, dFx, dFy, dFz;
        if constexpr (HLL) {
            // HLL face fluxes G = wl G(UL) + wr G(UR) + wd (UR - UL), the
            // weights from the signal speeds of the two cells of each face;
            // physical fluxes along d: N -> F_d, F_k -> c^2 P_kd (the
            // pressures here already hold c^2 P)
            const float c = A.c;
            const HllW wxm = hll_weights(lxmL, lxpL, lcur.xm, lcur.xp, c);
            const HllW wxp = hll_weights(lcur.xm, lcur.xp, lxmR, lxpR, c);
            const HllW wym = hll_weights(lymD, lypD, lcur.ym, lcur.yp, c);
            const HllW wyp = hll_weights(lcur.ym, lcur.yp, lymU, lypU, c);
            const HllW wzm = wz_prev;
            const HllW wzp = hll_weights(lcur.zm, lcur.zp, lnxt.zm, lnxt.zp, c);
            wz_prev = wzp;
            auto face = [](const HllW &w, float gL, float gR, float uL, float uR) {
                return w.wl * gL + w.wr * gR + w.wd * (uR - uL);
            };
            dN = (face(wxp, cur.Fx, FxR, cur.N, NR) - face(wxm, FxL, cur.Fx, NL, cur.N)) +
                 (face(wyp, cur.Fy, FyU, cur.N, NU) - face(wym, FyD, cur.Fy, ND, cur.N)) +
                 (face(wzp, cur.Fz, nxt.Fz, cur.N, nxt.N) -
                  face(wzm, prv.Fz, cur.Fz, prv.N, cur.N));
            dFx = (face(wxp, pcur.xx, PxxR, cur.Fx, FxR) -
                   face(wxm, PxxL, pcur.xx, FxL, cur.Fx)) +
                  (face(wyp, pcur.xy, PxyU, cur.Fx, FxU) -
                   face(wym, PxyD, pcur.xy, FxD, cur.Fx)) +
                  (face(wzp, pcur.xz, pnxt.xz, cur.Fx, nxt.Fx) -
                   face(wzm, pprv.xz, pcur.xz, prv.Fx, cur.Fx));
            dFy = (face(wxp, pcur.xy, PxyR, cur.Fy, FyR) -
                   face(wxm, PxyL, pcur.xy, FyL, cur.Fy)) +
                  (face(wyp, pcur.yy, PyyU, cur.Fy, FyU) -
                   face(wym, PyyD, pcur.yy, FyD, cur.Fy)) +
                  (face(wzp, pcur.yz, pnxt.yz, cur.Fy, nxt.Fy) -
                   face(wzm, pprv.yz, pcur.yz, prv.Fy, cur.Fy));
            dFz = (face(wxp, pcur.xz, PxzR, cur.Fz, FzR) -
                   face(wxm, PxzL, pcur.xz, FzL, cur.Fz)) +
                  (face(wyp, pcur.yz, PyzU, cur.Fz, FzU) -
                   face(wym, PyzD, pcur.yz, FzD, cur.Fz)) +
                  (face(wzp, pcur.zz, pnxt.zz, cur.Fz, nxt.Fz) -
                   face(wzm, pprv.zz, pcur.zz, prv.Fz, cur.Fz));
        } else {
            // sum over d of the LF face-flux differences G_{d,+1/2} - G_{d,-1/2}:
            //   N   : 1/2 (F_d[+] - F_d[-]) - c/2 (N[+] + N[-] - 2N)
            //   F_k : c^2/2 (P_kd[+] - P_kd[-]) - c/2 (F_k[+] + F_k[-] - 2F_k)
            const float hc = A.half_c, hc2 = A.half_c2;
            dN = 0.5f * ((FxR - FxL) + (FyU - FyD) + (nxt.Fz - prv.Fz)) -
                 hc * ((NL + NR) + (ND + NU) + (prv.N + nxt.N) - 6.0f * cur.N);
            dFx = hc2 * ((PxxR - PxxL) + (PxyU - PxyD) + (pnxt.xz - pprv.xz)) -
                  hc * ((FxL + FxR) + (FxD + FxU) + (prv.Fx + nxt.Fx) - 6.0f * cur.Fx);
            dFy = hc2 * ((PxyR - PxyL) + (PyyU - PyyD) + (pnxt.yz - pprv.yz)) -
                  hc * ((FyL + FyR) + (FyD + FyU) + (prv.Fy + nxt.Fy) - 6.0f * cur.Fy);
            dFz = hc2 * ((PxzR - PxzL) + (PyzU - PyzD) + (pnxt.zz - pprv.zz)) -
                  hc * ((FzL + FzR) + (FzD + FzU) + (prv.Fz + nxt.Fz) - 6.0f * cur.Fz);
        }

        // point sources of this plane (uniform walk over the sorted list)
        float S = 0.0f;
        const int zl = z - z0;
        while (sp < sp_end) {
            if (sp - buf_base >= buf_n) {          // uniform: refill the staging
                __syncthreads();
                buf_base = sp;
                buf_n = min(SRC_LDS, sp_end - sp);
                for (int i = tid; i < buf_n; i += KNT) {
                    s_skey[i] = A.src_key[buf_base + i];
                    s_srate[i] = A.src_rate[buf_base + i];
                }
                __syncthreads();
            }
            const int key = s_skey[sp - buf_base];
            if (key / KNT != zl) break;
            if (key - zl * KNT == tid) S += s_srate[sp - buf_base];
            ++sp;
        }

        float Nt = cur.N - A.k1 * dN + A.dt * S;
        float Fxt = cur.Fx - A.k1 * dFx;
        float Fyt = cur.Fy - A.k1 * dFy;
        float Fzt = cur.Fz - A.k1 * dFz;

        // photons through outflow faces: the face flux against the copied
        // image equals the edge cell's own normal flux
        float esc = 0.0f;
        if (A.any_outflow) {
            if (gx == 0 && A.bc[0] == RT_BC_OUTFLOW) esc -= cur.Fx;
            if (gx == A.nx - 1 && A.bc[1] == RT_BC_OUTFLOW) esc += cur.Fx;
            if (gy == 0 && A.bc[2] == RT_BC_OUTFLOW) esc -= cur.Fy;
            if (gy == A.ny - 1 && A.bc[3] == RT_BC_OUTFLOW) esc += cur.Fy;
            if (z == 0 && A.bc[4] == RT_BC_OUTFLOW) esc -= cur.Fz;
            if (z == A.nz - 1 && A.bc[5] == RT_BC_OUTFLOW) esc += cur.Fz;
        }

        // guards: N >= 0, |F| <= c N
        float flo = 0.0f;
        if (Nt < 0.0f) {
            flo = -Nt;
            Nt = 0.0f;
        }
        if (!(Nt > N_TINY)) {
            Fxt = Fyt = Fzt = 0.0f;
        } else {
            const float sN = A.inv_c * frcp(Nt);
            const float ux = Fxt * sN, uy = Fyt * sN, uz = Fzt * sN;
            const float u2 = ux * ux + uy * uy + uz * uz;
            if (u2 > 1.0f) {
                const float s = __builtin_amdgcn_rsqf(u2);
                Fxt *= s;
                Fyt *= s;
                Fzt *= s;
            }
        }

        // expansion over the step (operator split before Phi): dilution of
        // N and F, adiabatic cooling of the gas under the full chemistry
        float dil = 0.0f;
        if (A.expand) {
            dil = Nt * A.one_m_dil3;
            Nt *= A.dil3;
            Fxt *= A.dil3;
            Fyt *= A.dil3;
            Fzt *= A.dil3;
            if (A.chem == RT_CHEM_FULL) c_T *= A.dil2;
        }

        // per-cell operator Phi
        float Nn = Nt, xh = c_xh, Tc = c_T, pabs = 0.0f;
        int ncyc = 0;
        bool deferred = false;
        // Phi leaves a dark, fully neutral cell as it is, apart from the
        // temperature floor of the full chemistry; a wavefront of such cells
        // branches around the chemistry entirely
        const bool dark = !(Nt > 0.0f) && c_xh >= 1.0f;
        if (A.chem != RT_CHEM_OFF) {
            if (dark) {
                if (A.chem == RT_CHEM_FULL) Tc = rmax(c_T, A.T_floor);
            } else if (A.mixed && c_xh < A.xhi_thr) {
                deferred = true;   // FP64 chemistry, in the deferred kernel
            } else {
                float cR, cI;
                clump_f32(A.cl, c_nh, cR, cI);
                if (A.defer_stiff) {
                    // the adaptive operator's first sub-cycle: if it spans the
                    // step, this is the whole of Phi; otherwise the cell is
                    // stiff and goes to the deferred kernel
                    const RateSet rs = rates_f32(c_T, A.inv15kB);
                    const float tc = chem_timescale<float>(A.chem, Kf, rs, cR, cI, c_nh, Nt,
                                                           c_xh, 1.0f - c_xh, c_T);
                    // (written so that sub_eps = 0 defers every such cell,
                    // also one whose time scale overflowed to infinity)
                    if (!(A.sub_eps * tc >= A.dt)) {
                        deferred = true;
                    } else if (A.adaptive || A.nsub == 1) {
                        float xi = 1.0f - c_xh;
                        chem_sub<float>(A.chem, Kf, rs, cR, cI, c_nh, frcp(c_nh), A.dt, Nn, xh,
                                        xi, Tc, pabs);
                        ncyc = 1;
                    } else {
                        ncyc = chem_cell<float>(A.chem, A.nsub, 0, Kf, cR, cI, c_nh, Nn, xh, Tc,
                                                pabs);
                    }
                } else {
                    ncyc = chem_cell<float>(A.chem, A.nsub, A.adaptive, Kf, cR, cI, c_nh, Nn, xh,
                                            Tc, pabs);
                }
            }
        }
        if (A.chem != RT_CHEM_OFF && !deferred) {
            const float sc = (Nt > N_TINY) ? rmin(Nn * frcp(Nt), 1.0f) : 0.0f;
            Fxt *= sc;
            Fyt *= sc;
            Fzt *= sc;
        }

        {
            // lanes outside a ragged tile write to the sink, so that stores
            // are issued unconditionally too
            const uint32_t i = uint32_t(gy) * uint32_t(A.nx) + uint32_t(gx) + uint32_t(z) * plane;
            float *sink = A.sink + tid;
            store_out(active ? &A.No[i] : sink, Nn);
            store_out(active ? &A.Fxo[i] : sink, Fxt);
            store_out(active ? &A.Fyo[i] : sink, Fyt);
            store_out(active ? &A.Fzo[i] : sink, Fzt);
            store_out(active ? &A.xHI[i] : sink, xh);
            store_out(active ? &A.T[i] : sink, Tc);
        }
        if (A.defer) {
            // the word of plane z is kept by lane (z - z0) mod 64 and
            // stored once 64 planes are done: no store on every plane to
            // disturb the waits for the prefetched loads
            const unsigned long long m = __ballot(active && deferred);
            if (lx == ((z - z0) & 63)) mword = uint64_t(m);
        }
        if (active && !deferred) {
            // 0 * v is NaN exactly when v is infinite or NaN; inputs are
            // checked too, since the clamps of Phi would turn a NaN into a bound
            float z0 = 0.0f * Nn + 0.0f * Fxt + 0.0f * Fyt + 0.0f * Fzt + 0.0f * xh + 0.0f * Tc;
            z0 += 0.0f * cur.N + 0.0f * cur.Fx + 0.0f * cur.Fy + 0.0f * cur.Fz + 0.0f * c_xh +
                  0.0f * c_T + 0.0f * c_nh;
            const bool fin = z0 == 0.0f;
            n_bad += fin ? 0 : 1;
        }
        if (active && !deferred) {
            acc_xhi += double(xh);
            acc_nhxhi = fma(double(c_nh), double(xh), acc_nhxhi);
            acc_N += double(Nn);
            acc_abs += double(pabs);
        }
        {
            if (A.any_outflow) {
                double e = active ? double(esc) : 0.0;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
                if (lx == 0) s_acc[wave][4] += e;
            }
            if (__ballot(active && flo > 0.0f) != 0ull) {
                double f = active ? double(flo) : 0.0;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) f += __shfl_xor(f, off);
                if (lx == 0) s_acc[wave][5] += f;
            }
            if (A.expand) {
                double d = active ? double(dil) : 0.0;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
                if (lx == 0) s_acc[wave][6] += d;
            }
        }
        if (A.count_hist && A.chem != RT_CHEM_OFF) {
            const int bin = hist_bin(ncyc);
#pragma unroll
            for (int hb = 0; hb < 8; ++hb) {
                const unsigned long long m = __ballot(active && !deferred && bin == hb);
                if (lx == 0 && m) atomicAdd(&shist[hb], __popcll(m));
            }
        }

        // advance the z window (values loaded at least one plane ago)
        prv = cur;
        pprv = pcur;
        cur = nxt;
        pcur = pnxt;
        if constexpr (HLL) {
            lcur = lnxt;
        }
    };

    for (int z = z0; z < z1; z += 2) {
        plane_step(z, nx1, nx0, ha0, ha1, ch0, ch1, 0);
        if (z + 1 < z1) plane_step(z + 1, nx0, nx1, ha1, ha0, ch1, ch0, 1);
        if (A.defer && (((z + 2 - z0) & 63) == 0 || z + 2 >= z1)) {
            // one x-row per wave, 64 planes zb .. zb+63 of the chunk one per
            // lane, stored once they are done
            const int zb = z0 + ((z - z0) & ~63);
            if (gy < A.ny && zb + lx < z1) {
                const size_t w = (size_t(zb + lx) * A.ny + gy) * A.ntx + (x0 / TX);
                A.fp64_mask[w] = mword;
                if (mword) atomicOr(&A.group_mask[w >> 12], 1ull << ((w >> 6) & 63));
            }
            mword = 0;
        }
    }
    {
        double d[4] = {acc_xhi, acc_nhxhi, acc_N, acc_abs};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) d[j] += __shfl_xor(d[j], off);
        }
        if (lx == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) s_acc[wave][j] += d[j];
        }
    }

    // block reduction of the partial sums (fixed order, FP64)
    double v[1] = {double(n_bad)};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[0] += __shfl_xor(v[0], off);
    if (lx == 0) {
        sred[wave][R_XHI] = s_acc[wave][0];
        sred[wave][R_NHXHI] = s_acc[wave][1];
        sred[wave][R_NH] = 0.0;  // static: summed once at rt_init
        sred[wave][R_N] = s_acc[wave][2];
        sred[wave][R_ABS] = s_acc[wave][3] * A.vol;
        sred[wave][R_ESC] = s_acc[wave][4] * A.esc_scale;
        sred[wave][R_FLOOR] = s_acc[wave][5] * A.vol;
        sred[wave][R_NONFINITE] = v[0];
        sred[wave][R_FP64] = 0.0;       // FP64 cells are all deferred
        sred[wave][R_FALLBACK] = 0.0;   // so are the learned chemistry's cells
        sred[wave][R_LEARNED] = 0.0;
        sred[wave][R_RANGE] = 0.0;
        sred[wave][R_DILUTE] = s_acc[wave][6] * A.vol;
    }
    __syncthreads();
    if (tid < NRED) {
        double s = 0.0;
        if (tid < R_HIST0) {
#pragma unroll
            for (int w = 0; w < KNT / 64; ++w) s += sred[w][tid];
        } else {
            s = double(shist[tid - R_HIST0]);
        }
        A.partials[size_t(blockIdx.x) * NRED + tid] = s;
    }
}

// ------------------------------------------- deferred chemistry (dense)
// The cells the step marked in fp64_mask hold their transported N, F in the
// next buffer and their step-start xHI, T.  Each wavefront reads 64 mask
// words at a time (one per lane), gathers the marked cells of those 64 tile
// rows into a list in LDS and then takes them 64 at a time, one per lane,
// so that every lane of every batch works: the learned chemistry on the
// matrix cores (SURR, full chemistry only) with its photon accounting and
// acceptance test, and the exact operator Phi -- FP64 for the cells below
// the mixed form's threshold, FP32 otherwise -- for the cells it does not
// accept.  F is scaled by the photons left; the cell's share of the sums
// that the step left out is reduced per block in a fixed order.
constexpr int DEFER_THREADS = 256, DEFER_MAX_BLOCKS = 2048;
constexpr int DEFER_WAVES = DEFER_THREADS / 64;

// Learned chemistry of one cell from the network's standardised outputs
// (y0, y1): the predicted end state, the photons it absorbs (net
// ionisations + recombinations - collisional ionisations over dt at that
// state, so the photon budget stays exact) and the acceptance test: one
// backward-Euler step of length dt with every rate frozen at the predicted
// state (photoionisation by the photons left, case-B recombination,
// collisional ionisation and cooling at T') must land within surr_tol of
// the prediction (absolute in xHI, relative in T); the features must lie in
// the training range and the end state inside its bounds.  f: the raw log10
// features.  Returns true if accepted.
__device__ __forceinline__ bool surr_accept(const StepArgs &A, const float f[5], bool ood,
                                            float y0, float y1, float Nt, float c_xh, float c_T,
                                            float c_nh, float sR, float sI, float &Ns,
                                            float &xs, float &Ts, float &Ph)
{
    const float *nm = A.surr_norm;
    // the network predicts u = asinh(d / 1e-3) of the changes d of log10
    // xHI and log10 T; d = 1e-3 sinh u
    auto change = [](float u) {
        const float e = fexp2(u * 1.4426950408889634f);
        return 0.5e-3f * (e - frcp(e));
    };
    const float dx0 = change(y0 * nm[12] + nm[10]);
    const float dT0 = change(y1 * nm[13] + nm[11]);
    xs = fexp2((f[1] + dx0) * 3.321928094887362f);
    Ts = fexp2((f[2] + dT0) * 3.321928094887362f);
    const RateSet rs = rates_f32(Ts, A.inv15kB);
    const float x1 = 1.0f - xs, x0 = 1.0f - c_xh;
    const float nh2dt = c_nh * c_nh * A.dt;
    Ph = c_nh * (c_xh - xs) + sR * rs.alpha * nh2dt * x1 * x1 - rs.beta * nh2dt * x1 * xs;
    Ph = rmin(rmax(Ph, 0.0f), Nt);
    Ns = Nt - Ph;
    const float inv_nh = frcp(c_nh);
    const float xBE = (c_xh + sR * rs.alpha * c_nh * A.dt * x1 * x1) *
                      frcp(1.0f + sI * A.csig * A.dt * Ns + rs.beta * c_nh * A.dt * x1);
    const float rx = fabsf(xs - xBE);
    const float lu = A.dt * c_nh * (x1 * x1 * sR * rs.crb + x1 * xs * rs.cci) *
                     frcp((1.0f + x1) * Ts);
    const float TBE = ((1.0f + x0) * c_T + Ph * inv_nh * A.T_h) * frcp((1.0f + lu) * (1.0f + x1));
    const float rT = fabsf(Ts - TBE) * frcp(Ts);
    return !ood && xs >= 1e-12f && xs <= 1.0f && Ts >= A.T_floor && isfinite(Ts) &&
           rx <= A.surr_tol && rT <= A.surr_tol;
}

// ------------------------------------------- deferred cells, balanced
// The deferred kernels share the marked cells out evenly.  A counting pass
// gives every group of 64 mask words the rank of its first marked cell in
// word order: block b of the pass takes groups [256 b, 256 b + 256),
// counts their marked cells (only the groups whose bit is set hold any)
// and writes their offsets within the block (loc[g]) and the block's total;
// one block then turns the totals into exclusive block offsets
// (boff[nbc] = the number of marked cells), so that the rank of group g's
// first cell is boff[g / 256] + loc[g].  Wavefront k of a deferred kernel
// takes the cells of ranks [k CHUNK, (k + 1) CHUNK), then the chunk a grid
// further on: every wavefront gets the same number of cells however they
// cluster, and which wavefront takes which cell depends only on the mask.
constexpr int CHUNK = 256;          // cells per chunk: four batches of 64
constexpr int GPB = 256;            // groups per counting block
constexpr int GPW = 16;             // groups per wavefront of the count and the compaction
constexpr int CNT_THREADS = GPB / GPW * 64;   // 16 wavefronts: more loads in flight
constexpr int SCAN_THREADS = 1024;

__host__ __device__ inline uint64_t count_blocks(uint64_t nwords)
{
    return (mask_groups(nwords) + GPB - 1) / GPB;
}

// Offsets of the groups of src, see above; loc: ngroups entries, boff:
// count_blocks + 1 (the totals here, turned into offsets by
// block_offsets_kernel).  With copy, the words of the groups whose bit is
// set are also copied there.
__global__ __launch_bounds__(CNT_THREADS) void mask_count_kernel(const StepArgs A,
                                                                 const uint64_t *src,
                                                                 uint64_t *copy, uint64_t nwords,
                                                                 uint32_t *loc, uint32_t *boff)
{
    __shared__ uint32_t s_cnt[GPB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint64_t ngroups = mask_groups(nwords);
    const uint64_t g0 = uint64_t(blockIdx.x) * GPB + uint64_t(wave) * GPW;   // 16-aligned
    if (lane < GPW) s_cnt[wave * GPW + lane] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint64_t bits = g0 < ngroups ? (A.group_mask[g0 >> 6] >> (g0 & 63)) & ((1ull << GPW) - 1ull)
                                 : 0ull;
    while (bits) {
        // up to four marked groups at a time, their loads in flight together
        int gi[4];
        uint64_t wd[4];
        int n = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            gi[j] = bits ? __builtin_ctzll(bits) : 0;
            n += bits ? 1 : 0;
            bits &= bits ? bits - 1ull : 0ull;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t w = (g0 + uint64_t(gi[j])) * 64 + uint64_t(lane);
            wd[j] = (j < n && w < nwords) ? src[w] : 0ull;
            if (copy && j < n && w < nwords) copy[w] = wd[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int c = __popcll(wd[j]);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
            if (lane == 0 && j < n) s_cnt[wave * GPW + gi[j]] = uint32_t(c);
        }
    }
    __syncthreads();
    // exclusive scan of the block's 256 counts (one per thread of the first
    // four wavefronts)
    const uint32_t mine = t < GPB ? s_cnt[t] : 0u;
    uint32_t incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    __shared__ uint32_t s_wsum[GPB / 64];
    if (t < GPB && lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    if (t < GPB) {
        uint32_t before = 0;
        for (int w2 = 0; w2 < wave; ++w2) before += s_wsum[w2];
        const uint64_t g = uint64_t(blockIdx.x) * GPB + uint64_t(t);
        if (g < ngroups) loc[g] = before + incl - mine;
        if (t == GPB - 1) boff[blockIdx.x] = before + incl;
    }
}

// boff[0 .. nb) block totals -> exclusive offsets, boff[nb] = their sum.
__global__ __launch_bounds__(SCAN_THREADS) void block_offsets_kernel(uint32_t *boff, int nb)
{
    __shared__ uint32_t s[SCAN_THREADS];
    const int t = threadIdx.x;
    const int per = (nb + SCAN_THREADS - 1) / SCAN_THREADS;
    const int lo = t * per, hi = lo + per < nb ? lo + per : nb;
    uint32_t sum = 0;
    for (int i = lo; i < hi; ++i) sum += boff[i];
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {   // inclusive scan of the run sums
        const uint32_t v = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    uint32_t run = s[t] - sum;
    for (int i = lo; i < hi; ++i) {
        const uint32_t c = boff[i];
        boff[i] = run;
        run += c;
    }
    if (t == SCAN_THREADS - 1) boff[nb] = s[t];
}

// The marked cells of src as a dense list in word order: cells[rank] =
// linear cell index, ranks from loc and boff (mask_count_kernel and
// block_offsets_kernel on the same src first).  Same blocks as the count.
__global__ __launch_bounds__(CNT_THREADS) void mask_compact_kernel(const StepArgs A,
                                                                   const uint64_t *src,
                                                                   uint64_t nwords,
                                                                   const uint32_t *loc,
                                                                   const uint32_t *boff,
                                                                   uint32_t *cells)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t ngroups = mask_groups(nwords);
    const uint64_t g0 = uint64_t(blockIdx.x) * GPB + uint64_t(wave) * GPW;   // 16-aligned
    const uint32_t bbase = boff[blockIdx.x];
    uint64_t bits = g0 < ngroups ? (A.group_mask[g0 >> 6] >> (g0 & 63)) & ((1ull << GPW) - 1ull)
                                 : 0ull;
    while (bits) {
        int gi[4];
        uint64_t wd[4];
        int n = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            gi[j] = bits ? __builtin_ctzll(bits) : 0;
            n += bits ? 1 : 0;
            bits &= bits ? bits - 1ull : 0ull;
        }
        uint32_t gl[4];   // the groups' offsets within the block, loaded with the words
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t w = (g0 + uint64_t(gi[j])) * 64 + uint64_t(lane);
            wd[j] = (j < n && w < nwords) ? src[w] : 0ull;
            gl[j] = loc[g0 + uint64_t(gi[j])];   // gi[j] = 0 past n: group g0, which exists
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j >= n) break;
            const uint64_t g = g0 + uint64_t(gi[j]);
            const int cnt = __popcll(wd[j]);
            int incl = cnt, most = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off);
                if (lane >= off) incl += v;
                most = max(most, __shfl_xor(most, off));
            }
            const uint32_t gbase = bbase + gl[j];
            const uint64_t w = g * 64 + uint64_t(lane);
            const uint32_t cell0 = uint32_t(w / uint64_t(A.ntx)) * uint32_t(A.nx) +
                                   uint32_t(w % uint64_t(A.ntx)) * TX;
            const uint64_t nonzero = __ballot(wd[j] != 0ull);
            if (uint32_t(__popcll(nonzero)) < uint32_t(most)) {
                // few marked words, densely marked: all lanes store one word
                // at a time, lane l its bit l (ranks from the bits below it)
                const uint64_t below = (1ull << lane) - 1ull;
                for (uint64_t nz = nonzero; nz; nz &= nz - 1ull) {
                    const int k = __builtin_ctzll(nz);
                    const uint64_t wk = __shfl(wd[j], k);
                    const uint32_t c0 = __shfl(cell0, k);
                    const uint32_t rk = gbase + uint32_t(__shfl(incl - cnt, k));
                    if ((wk >> lane) & 1ull) cells[rk + uint32_t(__popcll(wk & below))] = c0 + uint32_t(lane);
                }
            } else {
                // sparsely marked words: each lane stores its own bits
                uint32_t r = gbase + uint32_t(incl - cnt);
                for (uint64_t m = wd[j]; m; m &= m - 1ull) cells[r++] = cell0 + uint32_t(__builtin_ctzll(m));
            }
        }
    }
}

// The cells of this wavefront's chunks of the dense list, four batches of
// 64 per chunk: `batch(cell, valid)` on all lanes at once.
template <typename F>
__device__ __forceinline__ void marked_chunks(const uint64_t nwords, const uint32_t *boff,
                                              const uint32_t *cells, F &&batch)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t total = boff[count_blocks(nwords)];
    const uint32_t nchunks = (total + CHUNK - 1) / CHUNK;
    const uint32_t waves = gridDim.x * DEFER_WAVES;
    for (uint32_t k = blockIdx.x * DEFER_WAVES + wave; k < nchunks; k += waves) {
        const uint32_t c0 = k * CHUNK, c1 = c0 + CHUNK < total ? c0 + CHUNK : total;
        // the chunk's cell indices first, all four loads in flight together
        uint32_t idx[CHUNK / 64];
#pragma unroll
        for (int q = 0; q < CHUNK / 64; ++q) {
            const uint32_t r = c0 + uint32_t(q * 64 + lane);
            idx[q] = r < c1 ? cells[r] : 0u;
        }
#pragma unroll 1
        for (int q = 0; q < CHUNK / 64; ++q) {
            const uint32_t b0 = c0 + uint32_t(q * 64);
            if (b0 >= c1) break;
            batch(idx[q], b0 + uint32_t(lane) < c1);
        }
    }
}

// Per-block partial row of the deferred kernels' sums, in a fixed order.
__device__ __forceinline__ void defer_partials(const StepArgs &A, int row, double (*sred)[NRED],
                                               const int *shist, double v[9], int lane,
                                               int wave, int tid)
{
#pragma unroll
    for (int j = 0; j < 9; ++j) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off);
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NRED; ++j) sred[wave][j] = 0.0;
        sred[wave][R_XHI] = v[0];
        sred[wave][R_NHXHI] = v[1];
        sred[wave][R_N] = v[2];
        sred[wave][R_ABS] = v[3] * A.vol;
        sred[wave][R_NONFINITE] = v[4];
        sred[wave][R_FP64] = v[5];
        sred[wave][R_FALLBACK] = v[6];
        sred[wave][R_LEARNED] = v[7];
        sred[wave][R_RANGE] = v[8];
    }
    __syncthreads();
    if (tid < NRED) {
        double sum = 0.0;
        if (tid < R_HIST0) {
#pragma unroll
            for (int w = 0; w < DEFER_WAVES; ++w) sum += sred[w][tid];
        } else {
            sum = double(shist[tid - R_HIST0]);
        }
        A.partials[size_t(row) * NRED + tid] = sum;
    }
}

// The exact operator Phi of the cells still marked: FP64 below the mixed
// form's threshold, FP32 otherwise.  Partial rows from A.nblocks + row0.
__global__ __launch_bounds__(DEFER_THREADS) void defer_chem_kernel(StepArgs A, uint64_t nwords,
                                                                   const uint32_t *boff,
                                                                   const uint32_t *cells, int row0)
{
    __shared__ double sred[DEFER_WAVES][NRED];
    __shared__ int shist[8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 8) shist[tid] = 0;
    __syncthreads();
    const ChemK<double> Kd{A.dt_d,      A.dt_d / double(A.nsub), A.csig_d,   A.T_h_d,
                           A.T_floor_d, A.sub_eps_d,             A.inv15kB_d};
    const ChemK<float> Kf{A.dt,      A.dt / float(A.nsub), A.csig,   A.T_h,
                          A.T_floor, A.sub_eps,            A.inv15kB};
    double acc_xhi = 0.0, acc_nhxhi = 0.0, acc_N = 0.0, acc_abs = 0.0;
    int n_bad = 0, n_fp64 = 0;
    marked_chunks(nwords, boff, cells, [&](uint32_t i, bool valid) {
        float Nt = 0.0f, Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
        float c_xh = 1.0f, c_T = 1.0e4f, c_nh = 1.0f;
        if (valid) {
            Nt = A.No[i];
            Fx = A.Fxo[i];
            Fy = A.Fyo[i];
            Fz = A.Fzo[i];
            c_xh = A.xHI[i];
            c_T = A.T[i];
            c_nh = A.nH[i];
        }
        float Nn = Nt, xh = c_xh, Tc = c_T;
        double pabs = 0.0;
        int ncyc = 0;
        if (valid) {
            if (A.mixed && c_xh < A.xhi_thr) {
                double Nd = Nt, xd = c_xh, Td = c_T, ad = 0.0, dR, dI;
                clump_f64(A.cld, double(c_nh), dR, dI);
                ncyc = chem_cell<double>(A.chem, A.nsub, A.adaptive, Kd, dR, dI, double(c_nh), Nd,
                                         xd, Td, ad);
                Nn = float(Nd);
                xh = float(xd);
                Tc = float(Td);
                pabs = ad;
                n_fp64 += 1;
            } else {
                float cR, cI, pab = 0.0f;
                clump_f32(A.cl, c_nh, cR, cI);
                ncyc = chem_cell<float>(A.chem, A.nsub, A.adaptive, Kf, cR, cI, c_nh, Nn, xh, Tc,
                                        pab);
                pabs = pab;
            }
            const float sc = (Nt > N_TINY) ? rmin(Nn * frcp(Nt), 1.0f) : 0.0f;
            store_out(&A.No[i], Nn);
            store_out(&A.Fxo[i], Fx * sc);
            store_out(&A.Fyo[i], Fy * sc);
            store_out(&A.Fzo[i], Fz * sc);
            store_out(&A.xHI[i], xh);
            store_out(&A.T[i], Tc);
            float z0v = 0.0f * Nn + 0.0f * Fx + 0.0f * Fy + 0.0f * Fz + 0.0f * xh + 0.0f * Tc;
            z0v += 0.0f * Nt + 0.0f * c_xh + 0.0f * c_T + 0.0f * c_nh;
            n_bad += z0v == 0.0f ? 0 : 1;
            acc_xhi += double(xh);
            acc_nhxhi = fma(double(c_nh), double(xh), acc_nhxhi);
            acc_N += double(Nn);
            acc_abs += pabs;
        }
        if (A.count_hist) {
            const int bin = hist_bin(ncyc);
#pragma unroll
            for (int hb = 0; hb < 8; ++hb) {
                const unsigned long long hm = __ballot(valid && bin == hb);
                if (lane == 0 && hm) atomicAdd(&shist[hb], __popcll(hm));
            }
        }
    });
    double v[9] = {acc_xhi, acc_nhxhi, acc_N, acc_abs, double(n_bad), double(n_fp64), 0.0, 0.0,
                   0.0};
    defer_partials(A, A.nblocks + row0 + int(blockIdx.x), sred, shist, v, lane, wave, tid);
}

// The learned chemistry of the marked cells, on the matrix cores: each
// wavefront gathers the marked cells of 64 mask words and runs the network
// on them 64 at a time; a cell whose prediction passes surr_accept takes it,
// a rejected cell stays marked (the word is written back with only those
// bits) for defer_chem_kernel, which then runs the exact operator on the
// rejected cells alone, in dense wavefronts.  Partial rows from A.nblocks.
__global__ __launch_bounds__(DEFER_THREADS) void surr_chem_kernel(StepArgs A, uint64_t nwords,
                                                                  const uint32_t *boff,
                                                                  const uint32_t *cells,
                                                                  uint64_t *rejected)
{
    __shared__ __attribute__((aligned(16))) __bf16 s_pk[PK_FWD * 8];
    __shared__ float s_bias[SURR_NBIAS];
    __shared__ double sred[DEFER_WAVES][NRED];
    __shared__ int shist[8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 8) shist[tid] = 0;
    for (int i = tid; i < PK_FWD; i += DEFER_THREADS)
        reinterpret_cast<uint4 *>(s_pk)[i] = reinterpret_cast<const uint4 *>(A.surr_pk)[i];
    for (int i = tid; i < SURR_NBIAS; i += DEFER_THREADS) s_bias[i] = A.surr_bias[i];
    __syncthreads();
    double acc_xhi = 0.0, acc_nhxhi = 0.0, acc_N = 0.0, acc_abs = 0.0;
    int n_bad = 0, n_fb = 0, n_net = 0, n_range = 0;
    const MlpBias mb{s_bias, s_bias + 64, s_bias + 128, s_bias + 192};
    const float *nm = A.surr_norm;
    marked_chunks(nwords, boff, cells, [&](uint32_t i, bool valid) {
        float Nt = 0.0f, c_xh = 1.0f, c_T = 1.0e4f, c_nh = 1.0f;
        if (valid) {
            Nt = A.No[i];
            c_xh = A.xHI[i];
            c_T = A.T[i];
            c_nh = A.nH[i];
        }
        const float LOG10_2 = 0.301029995664f;
        float f[5] = {LOG10_2 * flog2(c_nh), LOG10_2 * flog2(rmax(c_xh, 1e-30f)),
                      LOG10_2 * flog2(c_T), LOG10_2 * flog2(rmax(Nt, 1e-30f)), A.log10_dt};
        bool ood = !(c_nh > 0.0f && c_T > 0.0f);
        float sv[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            ood = ood || !(f[k] >= nm[14 + k] && f[k] <= nm[19 + k]);
            sv[k] = valid ? (f[k] - nm[k]) * frcp(nm[5 + k]) : 0.0f;
        }
        float y0, y1;
        mlp_predict64(reinterpret_cast<const bf16x8 *>(s_pk), mb, sv, y0, y1);
        float cR, cI, Ns, xs, Ts, Ph;
        clump_f32(A.cl, c_nh, cR, cI);
        const bool ok = valid && surr_accept(A, f, ood, y0, y1, Nt, c_xh, c_T, c_nh, cR, cI, Ns,
                                             xs, Ts, Ph);
        if (ok) {
            const float sc = (Nt > N_TINY) ? rmin(Ns * frcp(Nt), 1.0f) : 0.0f;
            const float Fx = A.Fxo[i], Fy = A.Fyo[i], Fz = A.Fzo[i];
            store_out(&A.No[i], Ns);
            store_out(&A.Fxo[i], Fx * sc);
            store_out(&A.Fyo[i], Fy * sc);
            store_out(&A.Fzo[i], Fz * sc);
            store_out(&A.xHI[i], xs);
            store_out(&A.T[i], Ts);
            float z0v = 0.0f * Ns + 0.0f * Fx + 0.0f * Fy + 0.0f * Fz + 0.0f * xs + 0.0f * Ts;
            z0v += 0.0f * Nt + 0.0f * c_xh + 0.0f * c_T + 0.0f * c_nh;
            n_bad += z0v == 0.0f ? 0 : 1;
            n_net += 1;
            acc_xhi += double(xs);
            acc_nhxhi = fma(double(c_nh), double(xs), acc_nhxhi);
            acc_N += double(Ns);
            acc_abs += double(Ph);
        } else if (valid) {
            n_fb += 1;
            n_range += ood ? 1 : 0;
        }
        // Accepted cells leave the copy of the mask that the exact kernel
        // reads next (`rejected`; the mask this kernel reads stays as it is),
        // so that the exact kernel takes only the rejected ones.  The
        // batch's cells come in word order: the lanes of one word OR their
        // bits together (a segmented scan) and the word's last lane clears
        // them with one atomic.
        const uint32_t x = i % uint32_t(A.nx);
        // (lanes without a cell take a word index no cell has)
        const uint64_t wd = valid ? uint64_t(i / uint32_t(A.nx)) * uint64_t(A.ntx) + uint64_t(x / TX)
                                  : ~0ull;
        uint64_t bits = ok ? (1ull << (x & 63)) : 0ull;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t vb = __shfl_up(bits, off);
            const uint64_t vw = __shfl_up(wd, off);
            if (lane >= off && vw == wd) bits |= vb;
        }
        const uint64_t next = __shfl_down(wd, 1);
        const bool last = valid && (lane == 63 || next != wd);
        if (last && bits) atomicAnd(reinterpret_cast<unsigned long long *>(&rejected[wd]),
                                    ~(unsigned long long)bits);
        if (A.count_hist) {
            // accepted cells count in the first bin; the exact kernel counts
            // the rejected ones
            const unsigned long long hm = __ballot(ok);
            if (lane == 0 && hm) atomicAdd(&shist[0], __popcll(hm));
        }
    });
    double v[9] = {acc_xhi, acc_nhxhi, acc_N, acc_abs, double(n_bad), 0.0, double(n_fb),
                   double(n_net), double(n_range)};
    defer_partials(A, A.nblocks + int(blockIdx.x), sred, shist, v, lane, wave, tid);
}

size_t defer_offsets_size(uint64_t nwords)
{
    return size_t(mask_groups(nwords) + count_blocks(nwords) + 1);
}

// Blocks of the deferred kernels: enough wavefronts to fill the chip
// whatever the number of marked cells (they share the chunks of CHUNK
// cells), fewer on small grids.
int defer_chem_blocks(uint64_t nwords)
{
    const uint64_t want = (nwords * 64 / CHUNK + DEFER_WAVES - 1) / DEFER_WAVES;
    return int(want < 1 ? 1 : (want > DEFER_MAX_BLOCKS ? DEFER_MAX_BLOCKS : want));
}

hipError_t launch_defer_chem(const StepArgs &a, uint64_t nwords, int nb2, uint32_t *goff,
                             uint32_t *cells, uint64_t *mask2, hipStream_t s)
{
    const uint64_t nbc = count_blocks(nwords);
    uint32_t *loc = goff, *boff = goff + mask_groups(nwords);
    // the marked cells of `mask` into the dense list (copying the marked
    // groups' words to `copy` on the way when it is given)
    auto list = [&](const uint64_t *mask, uint64_t *copy) {
        hipLaunchKernelGGL(mask_count_kernel, dim3(unsigned(nbc)), dim3(CNT_THREADS), 0, s, a, mask, copy,
                           nwords, loc, boff);
        hipLaunchKernelGGL(block_offsets_kernel, dim3(1), dim3(SCAN_THREADS), 0, s, boff,
                           int(nbc));
        hipLaunchKernelGGL(mask_compact_kernel, dim3(unsigned(nbc)), dim3(CNT_THREADS), 0, s, a, mask,
                           nwords, static_cast<const uint32_t *>(loc),
                           static_cast<const uint32_t *>(boff), cells);
    };
    const uint64_t *exact_mask = a.fp64_mask;
    int row0 = 0;
    if (a.surr && a.chem == RT_CHEM_FULL) {
        list(a.fp64_mask, mask2);
        hipLaunchKernelGGL(surr_chem_kernel, dim3(nb2), dim3(DEFER_THREADS), 0, s, a, nwords,
                           static_cast<const uint32_t *>(boff), static_cast<const uint32_t *>(cells),
                           mask2);
        exact_mask = mask2;
        row0 = nb2;
    }
    list(exact_mask, nullptr);
    hipLaunchKernelGGL(defer_chem_kernel, dim3(nb2), dim3(DEFER_THREADS), 0, s, a, nwords,
                       static_cast<const uint32_t *>(boff), static_cast<const uint32_t *>(cells),
                       row0);
    return hipGetLastError();
}

// ---------------------------------------------- finalisation (one block)
// mode 0: a step -- ACC_CUR = sums, ACC_CUM += sums.
// mode 1: initial state -- ACC_CUR = sums, ACC_CUM = 0.
// Each thread sums a fixed strided subset of the block partials in FP64,
// then wavefronts and finally one thread per value combine them in a fixed
// order: the result does not depend on timing.
constexpr int FIN_THREADS = 1024;

__global__ __launch_bounds__(FIN_THREADS) void finalize_kernel(const double *__restrict__ part,
                                                               int nb, double *__restrict__ acc,
                                                               int mode, double tau_coef,
                                                               double nh_sum,
                                                               uint64_t *__restrict__ clear,
                                                               int nclear)
{
    // the deferred kernels' group bits of this step, cleared for the next
    for (int i = threadIdx.x; i < nclear; i += FIN_THREADS) clear[i] = 0ull;
    __shared__ double s[FIN_THREADS / 64][NRED];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double v[NRED];
#pragma unroll
    for (int j = 0; j < NRED; ++j) v[j] = 0.0;
    for (int b = t; b < nb; b += FIN_THREADS) {
        const double *p = part + size_t(b) * NRED;
#pragma unroll
        for (int j = 0; j < NRED; ++j) v[j] += p[j];
    }
#pragma unroll
    for (int j = 0; j < NRED; ++j) {
        double x = v[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) s[wave][j] = x;
    }
    __syncthreads();
    if (t < NRED) {
        double x = 0.0;
#pragma unroll
        for (int w = 0; w < FIN_THREADS / 64; ++w) x += s[w][t];
        acc[ACC_CUR + t] = x;
        if (mode == 0)
            acc[ACC_CUM + t] += x;
        else
            acc[ACC_CUM + t] = 0.0;
        // Thomson depth: c sigma_T dt <nH (1 - xHI)> after the step
        if (t == R_NHXHI) {
            if (mode == 0)
                acc[ACC_CUM + ACC_TAU] += tau_coef * (nh_sum - x);
            else
                acc[ACC_CUM + ACC_TAU] = 0.0;
        }
    }
}

// First level for large grids: FIN1_BLOCKS blocks, each summing a contiguous
// range of block partials in a fixed order (strided per thread, then the
// wavefronts and the block), so that finalize_kernel only combines
// FIN1_BLOCKS rows.  One block reading every partial is latency-bound.
__global__ __launch_bounds__(256) void finalize_partial_kernel(const double *__restrict__ part,
                                                               int nb,
                                                               double *__restrict__ out)
{
    __shared__ double s[4][NRED];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int per = (nb + int(gridDim.x) - 1) / int(gridDim.x);
    const int b0 = int(blockIdx.x) * per, b1 = min(nb, b0 + per);
    double v[NRED];
#pragma unroll
    for (int j = 0; j < NRED; ++j) v[j] = 0.0;
    for (int b = b0 + t; b < b1; b += 256) {
        const double *p = part + size_t(b) * NRED;
#pragma unroll
        for (int j = 0; j < NRED; ++j) v[j] += p[j];
    }
#pragma unroll
    for (int j = 0; j < NRED; ++j) {
        double x = v[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) s[wave][j] = x;
    }
    __syncthreads();
    if (t < NRED) out[size_t(blockIdx.x) * NRED + t] = ((s[0][t] + s[1][t]) + s[2][t]) + s[3][t];
}

// --------------------------------------- sums of a state (at rt_init)
__global__ __launch_bounds__(256) void state_sums_kernel(const float *__restrict__ N,
                                                         const float *__restrict__ xHI,
                                                         const float *__restrict__ nH,
                                                         uint32_t ncell,
                                                         double *__restrict__ part)
{
    __shared__ double s[4][256];
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    // 64-bit index: with ncell just below 2^32 a 32-bit index would wrap
    // past the end and never leave the loop
    const uint64_t stride = uint64_t(gridDim.x) * 256u;
    for (uint64_t i = uint64_t(blockIdx.x) * 256u + t; i < ncell; i += stride) {
        const double x = xHI[i], n = nH[i];
        a0 += x;
        a1 += n * x;
        a2 += n;
        a3 += N[i];
    }
    s[0][t] = a0;
    s[1][t] = a1;
    s[2][t] = a2;
    s[3][t] = a3;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int j = 0; j < 4; ++j) s[j][t] += s[j][t + w];
        __syncthreads();
    }
    if (t < NRED) {
        double v = 0.0;
        if (t == R_XHI) v = s[0][0];
        if (t == R_NHXHI) v = s[1][0];
        if (t == R_NH) v = s[2][0];
        if (t == R_N) v = s[3][0];
        part[size_t(blockIdx.x) * NRED + t] = v;
    }
}

int state_sums_blocks(uint32_t ncell)
{
    uint32_t b = (ncell + 255u) / 256u;
    return int(b < 1024u ? (b > 0 ? b : 1) : 1024u);
}

hipError_t launch_step(const StepArgs &a, hipStream_t s)
{
    const dim3 g(a.nblocks), b(a.big ? NTHREADS_LF : (a.hll ? NTHREADS_HLL : NTHREADS));
    if (a.hll)
        hipLaunchKernelGGL((m1_step_kernel<true, false>), g, b, 0, s, a);
    else if (a.big)
        hipLaunchKernelGGL((m1_step_kernel<false, true>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((m1_step_kernel<false, false>), g, b, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nblocks, double *scratch, double *acc,
                           int mode, double tau_coef, double nh_sum, hipStream_t s,
                           uint64_t *clear, int nclear)
{
    if (nblocks > FIN1_MIN) {
        hipLaunchKernelGGL(finalize_partial_kernel, dim3(FIN1_BLOCKS), dim3(256), 0, s,
                           partials, nblocks, scratch);
        partials = scratch;
        nblocks = FIN1_BLOCKS;
    }
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(FIN_THREADS), 0, s, partials, nblocks,
                       acc, mode, tau_coef, nh_sum, clear, nclear);
    return hipGetLastError();
}

hipError_t launch_state_sums(const float *N, const float *xHI, const float *nH,
                             uint32_t ncell, double *partials, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(state_sums_kernel, dim3(nblocks), dim3(256), 0, s, N, xHI, nH, ncell,
                       partials);
    return hipGetLastError();
}

}  // namespace rtk
