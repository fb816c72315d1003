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
//   * the unsplit Lax-Friedrichs update, the point sources, the positivity
//     guards, the sub-cycled chemistry Phi and the FP64 global sums all
//     happen on values already in registers; each cell is read and written
//     exactly once;
//   * blocks are renumbered so that each XCD (blockIdx mod 8) receives a
//     contiguous run of neighbouring tiles and shares their halo rows in its
//     own L2.
#include <math.h>

#include "mlp_device.h"

#ifndef RT_M1_NT_STORES
#define RT_M1_NT_STORES 0
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
// Exact forms: at most 128 VGPRs so that two 512-thread blocks (4 waves per
// SIMD) share a CU; the surrogate form needs more and runs one block.
template <bool MIXED, bool SURR>
__global__ __launch_bounds__(NTHREADS, SURR ? 2 : 4) void m1_step_kernel(StepArgs A)
{
    constexpr int SW = TX + 2;
    __shared__ __attribute__((aligned(16))) __bf16 s_pk[SURR ? PK_FWD * 8 : 8];
    __shared__ float s_bias[SURR ? SURR_NBIAS : 1];
    __shared__ float sN[TY + 2][SW], sFx[TY + 2][SW], sFy[TY + 2][SW], sFz[TY + 2][SW];
    __shared__ float sPxx[TY + 2][SW], sPyy[TY + 2][SW], sPxy[TY + 2][SW];
    __shared__ float sPxz[TY + 2][SW], sPyz[TY + 2][SW];
    __shared__ double sred[NTHREADS / 64][NRED];

    const int tid = threadIdx.x;
    const int lx = tid & (TX - 1), ly = tid / TX;
    if (SURR) {
        // network operands to LDS (read by every plane; the first barrier of
        // the z loop orders these stores before any use)
        for (int i = tid; i < PK_FWD; i += NTHREADS)
            reinterpret_cast<uint4 *>(s_pk)[i] = reinterpret_cast<const uint4 *>(A.surr_pk)[i];
        for (int i = tid; i < SURR_NBIAS; i += NTHREADS) s_bias[i] = A.surr_bias[i];
    }

    // XCD-aware renumbering: blockIdx mod 8 selects the XCD; each XCD takes
    // a contiguous range of tiles (x fastest, then y, then the z chunk).
    const int b = blockIdx.x, nb = A.nblocks;
    const int q = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int tile = xcd * q + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int itx = tile % A.ntx;
    const int rest = tile / A.ntx;
    const int ity = rest % A.nty;
    const int izc = rest / A.nty;
    const int x0 = itx * TX, y0 = ity * TY;
    const int z0 = izc * A.zc;
    const int z1 = min(z0 + A.zc, A.nz);
    const int gx = x0 + lx, gy = y0 + ly;
    const bool active = gx < A.nx && gy < A.ny;
    const uint32_t plane = A.plane;

    // own column (boundary image for slots outside the grid)
    const Map1 mx = map_coord(gx, A.nx, A.bc[0], A.bc[1]);
    const Map1 my = map_coord(gy, A.ny, A.bc[2], A.bc[3]);
    const uint32_t col = uint32_t(my.idx) * uint32_t(A.nx) + uint32_t(mx.idx);

    // halo slot of this thread: rows y0-1 and y0+TY, columns x0-1 and x0+TX
    int hsx = 0, hsy = 0;
    const bool has_halo = tid < 2 * TX + 2 * TY;
    if (tid < TX) {
        hsy = 0;
        hsx = tid + 1;
    } else if (tid < 2 * TX) {
        hsy = TY + 1;
        hsx = tid - TX + 1;
    } else if (tid < 2 * TX + TY) {
        hsx = 0;
        hsy = tid - 2 * TX + 1;
    } else {
        hsx = TX + 1;
        hsy = tid - 2 * TX - TY + 1;
    }
    const Map1 hx = map_coord(x0 + hsx - 1, A.nx, A.bc[0], A.bc[1]);
    const Map1 hy = map_coord(y0 + hsy - 1, A.ny, A.bc[2], A.bc[3]);
    const uint32_t hcol = uint32_t(hy.idx) * uint32_t(A.nx) + uint32_t(hx.idx);

    // sources of this tile, sorted by plane
    int sp = A.src_ptr[tile];
    const int sp_end = A.src_ptr[tile + 1];

    // FP64 accumulators
    double acc_xhi = 0.0, acc_nhxhi = 0.0, acc_N = 0.0;
    double acc_abs = 0.0, acc_esc = 0.0, acc_floor = 0.0;
    int n_bad = 0, n_fp64 = 0, n_fb = 0;
    __shared__ int shist[8];
    if (tid < 8) shist[tid] = 0;

    const ChemK<float> Kf{A.dt, A.dt / float(A.nsub), A.csig, A.T_h, A.T_floor, A.sub_eps};
    const ChemK<double> Kd{A.dt_d, A.dt_d / double(A.nsub), A.csig_d, A.T_h_d, A.T_floor_d,
                           A.sub_eps_d};

    // prologue: plane z0-1 (boundary image if outside), plane z0, plane z0+1
    const Map1 mzm = map_coord(z0 - 1, A.nz, A.bc[4], A.bc[5]);
    Cell4 prv = load4(A, col + uint32_t(mzm.idx) * plane, mx.sign, my.sign, mzm.sign);
    Press pprv = closure(prv.N, prv.Fx, prv.Fy, prv.Fz, A.inv_c);
    Cell4 cur = load4(A, col + uint32_t(z0) * plane, mx.sign, my.sign, 1.0f);
    Press pcur = closure(cur.N, cur.Fx, cur.Fy, cur.Fz, A.inv_c);
    Map1 mzp = map_coord(z0 + 1, A.nz, A.bc[4], A.bc[5]);
    Cell4 nxt = load4(A, col + uint32_t(mzp.idx) * plane, mx.sign, my.sign, mzp.sign);
    Cell4 hal{0.f, 0.f, 0.f, 0.f};
    if (has_halo) hal = load4(A, hcol + uint32_t(z0) * plane, hx.sign, hy.sign, 1.0f);
    float c_xh = A.xHI[col + uint32_t(z0) * plane];
    float c_T = A.T[col + uint32_t(z0) * plane];
    float c_nh = A.nH[col + uint32_t(z0) * plane];

    for (int z = z0; z < z1; ++z) {
        // prefetch plane z+1 (halo, chemistry fields) and z+2 (own column)
        const bool more = z + 1 < z1;
        const int zn = more ? z + 1 : z;
        const Map1 mzq = map_coord(z + 2, A.nz, A.bc[4], A.bc[5]);
        Cell4 nx2 = nxt;
        if (more) nx2 = load4(A, col + uint32_t(mzq.idx) * plane, mx.sign, my.sign, mzq.sign);
        Cell4 hal2 = hal;
        if (has_halo && more) hal2 = load4(A, hcol + uint32_t(zn) * plane, hx.sign, hy.sign, 1.0f);
        const uint32_t inext = col + uint32_t(zn) * plane;
        const float n_xh = A.xHI[inext];
        const float n_T = A.T[inext];
        const float n_nh = A.nH[inext];

        // plane z into LDS: own cell and its halo
        {
            const int sy = ly + 1, sx = lx + 1;
            sN[sy][sx] = cur.N;
            sFx[sy][sx] = cur.Fx;
            sFy[sy][sx] = cur.Fy;
            sFz[sy][sx] = cur.Fz;
            sPxx[sy][sx] = pcur.xx;
            sPyy[sy][sx] = pcur.yy;
            sPxy[sy][sx] = pcur.xy;
            sPxz[sy][sx] = pcur.xz;
            sPyz[sy][sx] = pcur.yz;
        }
        if (has_halo) {
            const Press ph = closure(hal.N, hal.Fx, hal.Fy, hal.Fz, A.inv_c);
            sN[hsy][hsx] = hal.N;
            sFx[hsy][hsx] = hal.Fx;
            sFy[hsy][hsx] = hal.Fy;
            sFz[hsy][hsx] = hal.Fz;
            sPxx[hsy][hsx] = ph.xx;
            sPyy[hsy][hsx] = ph.yy;
            sPxy[hsy][hsx] = ph.xy;
            sPxz[hsy][hsx] = ph.xz;
            sPyz[hsy][hsx] = ph.yz;
        }
        __syncthreads();

        const Press pnxt = closure(nxt.N, nxt.Fx, nxt.Fy, nxt.Fz, A.inv_c);
        const int sy = ly + 1, sx = lx + 1;
        // neighbours: x-1 (L), x+1 (R), y-1 (D), y+1 (U), z-1 (prv), z+1 (nxt)
        const float NL = sN[sy][sx - 1], NR = sN[sy][sx + 1];
        const float ND = sN[sy - 1][sx], NU = sN[sy + 1][sx];
        const float FxL = sFx[sy][sx - 1], FxR = sFx[sy][sx + 1];
        const float FxD = sFx[sy - 1][sx], FxU = sFx[sy + 1][sx];
        const float FyL = sFy[sy][sx - 1], FyR = sFy[sy][sx + 1];
        const float FyD = sFy[sy - 1][sx], FyU = sFy[sy + 1][sx];
        const float FzL = sFz[sy][sx - 1], FzR = sFz[sy][sx + 1];
        const float FzD = sFz[sy - 1][sx], FzU = sFz[sy + 1][sx];
        const float PxxL = sPxx[sy][sx - 1], PxxR = sPxx[sy][sx + 1];
        const float PxyL = sPxy[sy][sx - 1], PxyR = sPxy[sy][sx + 1];
        const float PxzL = sPxz[sy][sx - 1], PxzR = sPxz[sy][sx + 1];
        const float PxyD = sPxy[sy - 1][sx], PxyU = sPxy[sy + 1][sx];
        const float PyyD = sPyy[sy - 1][sx], PyyU = sPyy[sy + 1][sx];
        const float PyzD = sPyz[sy - 1][sx], PyzU = sPyz[sy + 1][sx];
        __syncthreads();

        // sum over d of the LF face-flux differences G_{d,+1/2} - G_{d,-1/2}:
        //   N   : 1/2 (F_d[+] - F_d[-]) - c/2 (N[+] + N[-] - 2N)
        //   F_k : c^2/2 (P_kd[+] - P_kd[-]) - c/2 (F_k[+] + F_k[-] - 2F_k)
        const float hc = A.half_c, hc2 = A.half_c2;
        const float dN = 0.5f * ((FxR - FxL) + (FyU - FyD) + (nxt.Fz - prv.Fz)) -
                         hc * ((NL + NR) + (ND + NU) + (prv.N + nxt.N) - 6.0f * cur.N);
        const float dFx = hc2 * ((PxxR - PxxL) + (PxyU - PxyD) + (pnxt.xz - pprv.xz)) -
                          hc * ((FxL + FxR) + (FxD + FxU) + (prv.Fx + nxt.Fx) - 6.0f * cur.Fx);
        const float dFy = hc2 * ((PxyR - PxyL) + (PyyU - PyyD) + (pnxt.yz - pprv.yz)) -
                          hc * ((FyL + FyR) + (FyD + FyU) + (prv.Fy + nxt.Fy) - 6.0f * cur.Fy);
        const float dFz = hc2 * ((PxzR - PxzL) + (PyzU - PyzD) + (pnxt.zz - pprv.zz)) -
                          hc * ((FzL + FzR) + (FzD + FzU) + (prv.Fz + nxt.Fz) - 6.0f * cur.Fz);

        // point sources of this plane (uniform walk over the sorted list)
        float S = 0.0f;
        const int zl = z - z0;
        while (sp < sp_end) {
            const int key = A.src_key[sp];
            if (key / NTHREADS != zl) break;
            if (key - zl * NTHREADS == tid) S += A.src_rate[sp];
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

        // per-cell operator Phi
        float Nn = Nt, xh = c_xh, Tc = c_T;
        double pabs = 0.0;
        int ncyc = 0;
        bool used64 = false;
        bool fallback = true;
        if (SURR) {
            // learned Phi for the 64 cells of this wavefront (uniform control
            // flow: every lane takes part in the matrix products)
            const float *nm = A.surr_norm;
            const float LOG10_2 = 0.301029995664f;
            float f[5] = {LOG10_2 * flog2(c_nh), LOG10_2 * flog2(rmax(c_xh, 1e-30f)),
                          LOG10_2 * flog2(c_T), LOG10_2 * flog2(rmax(Nt, 1e-30f)), A.log10_dt};
            bool ood = !(c_nh > 0.0f && c_T > 0.0f);
            float sv[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                ood = ood || !(f[k] >= nm[14 + k] && f[k] <= nm[19 + k]);
                sv[k] = (f[k] - nm[k]) * frcp(nm[5 + k]);
            }
            const int lane = tid & 63;
            bf16x8 xa, xb;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                xa[k] = (__bf16)0.0f;
                xb[k] = (__bf16)0.0f;
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const float up = __shfl(sv[k], (lane + 32) & 63);
                if (lane < 32) {
                    xa[k] = (__bf16)sv[k];
                    xb[k] = (__bf16)up;
                }
            }
            const MlpBias mb{s_bias, s_bias + 64, s_bias + 128, s_bias + 192};
            const bf16x8 *spk = reinterpret_cast<const bf16x8 *>(s_pk);
            MlpFwd unused;
            float ya0, ya1, yb0, yb1;
            mlp_forward32<false>(spk, mb, xa, unused, ya0, ya1);
            mlp_forward32<false>(spk, mb, xb, unused, yb0, yb1);
            const float sb0 = __shfl(yb0, lane & 31), sb1 = __shfl(yb1, lane & 31);
            const float y0 = lane < 32 ? ya0 : sb0, y1 = lane < 32 ? ya1 : sb1;
            // decode: log10 xHI', log10 T'
            const float xs = fexp2((y0 * nm[12] + nm[10]) * 3.321928094887362f);
            float Ts = fexp2((y1 * nm[13] + nm[11]) * 3.321928094887362f);
            if (A.chem != RT_CHEM_FULL) Ts = c_T;
            // photons absorbed over dt: net ionisations + recombinations -
            // collisional ionisations at the predicted end state
            const RateSet rs = rates_f32(Ts, A.inv15kB);
            const float x1 = 1.0f - xs, x0 = 1.0f - c_xh;
            const float nh2dt = c_nh * c_nh * A.dt;
            float Ph = c_nh * (c_xh - xs) + rs.alpha * nh2dt * x1 * x1 - rs.beta * nh2dt * x1 * xs;
            Ph = rmin(rmax(Ph, 0.0f), Nt);
            const float Ns = Nt - Ph;
            // backward-Euler residuals of one step dt at the predicted end
            const float inv_nh = frcp(c_nh);
            const float rx = fabsf(Ph - A.csig * A.dt * Ns * c_nh * xs) * inv_nh;
            float rT = 0.0f;
            if (A.chem == RT_CHEM_FULL) {
                const float lu = A.dt * c_nh * (x1 * x1 * rs.crb + x1 * xs * rs.cci) *
                                 frcp((1.0f + x1) * Ts);
                const float TBE = ((1.0f + x0) * c_T + Ph * inv_nh * A.T_h) *
                                  frcp((1.0f + lu) * (1.0f + x1));
                rT = fabsf(Ts - TBE) * frcp(Ts);
            }
            const bool ok = A.chem == RT_CHEM_FULL && !ood && xs >= 1e-12f && xs <= 1.0f &&
                            Ts >= A.T_floor && isfinite(Ts) && rx <= A.surr_tol &&
                            rT <= A.surr_tol;
            if (ok) {
                fallback = false;
                Nn = Ns;
                xh = xs;
                Tc = Ts;
                pabs = Ph;
            }
        }
        // Phi leaves a dark, fully neutral cell exactly as it is; a
        // wavefront of such cells branches around the chemistry entirely
        const bool dark = !(Nt > 0.0f) && c_xh >= 1.0f;
        if (A.chem != RT_CHEM_OFF && fallback && !dark) {
            if (MIXED && c_xh < A.xhi_thr) {
                double Nd = Nt, xd = c_xh, Td = c_T, ad = 0.0;
                ncyc = chem_cell<double>(A.chem, A.nsub, A.adaptive, A.inv15kB, Kd,
                                         double(c_nh), Nd, xd, Td, ad);
                Nn = float(Nd);
                xh = float(xd);
                Tc = float(Td);
                pabs = ad;
                used64 = true;
            } else {
                float af = 0.0f;
                ncyc = chem_cell<float>(A.chem, A.nsub, A.adaptive, A.inv15kB, Kf, c_nh, Nn,
                                        xh, Tc, af);
                pabs = af;
            }
        }
        if (A.chem != RT_CHEM_OFF) {
            const float sc = (Nt > N_TINY) ? rmin(Nn * frcp(Nt), 1.0f) : 0.0f;
            Fxt *= sc;
            Fyt *= sc;
            Fzt *= sc;
        }

        if (active) {
            const uint32_t i = uint32_t(gy) * uint32_t(A.nx) + uint32_t(gx) + uint32_t(z) * plane;
            store_out(&A.No[i], Nn);
            store_out(&A.Fxo[i], Fxt);
            store_out(&A.Fyo[i], Fyt);
            store_out(&A.Fzo[i], Fzt);
            store_out(&A.xHI[i], xh);
            store_out(&A.T[i], Tc);
            acc_xhi += double(xh);
            acc_nhxhi = fma(double(c_nh), double(xh), acc_nhxhi);
            acc_N += double(Nn);
            acc_abs += pabs;
            if (A.any_outflow) acc_esc += double(esc);
            if (flo > 0.0f) acc_floor += double(flo);
            // 0 * v is NaN exactly when v is infinite or NaN; inputs are
            // checked too, since the clamps of Phi would turn a NaN into a bound
            float z0 = 0.0f * Nn + 0.0f * Fxt + 0.0f * Fyt + 0.0f * Fzt + 0.0f * xh + 0.0f * Tc;
            z0 += 0.0f * cur.N + 0.0f * cur.Fx + 0.0f * cur.Fy + 0.0f * cur.Fz + 0.0f * c_xh +
                  0.0f * c_T + 0.0f * c_nh;
            const bool fin = z0 == 0.0f;
            n_bad += fin ? 0 : 1;
            n_fp64 += used64 ? 1 : 0;
            n_fb += (SURR && fallback && A.chem != RT_CHEM_OFF) ? 1 : 0;
        }
        if ((A.adaptive || SURR) && A.chem != RT_CHEM_OFF) {
            const int bin = hist_bin(ncyc);
#pragma unroll
            for (int hb = 0; hb < 8; ++hb) {
                const unsigned long long m = __ballot(active && fallback && bin == hb);
                if (lx == 0 && m) atomicAdd(&shist[hb], __popcll(m));
            }
        }

        // rotate the z pipeline
        prv = cur;
        pprv = pcur;
        cur = nxt;
        pcur = pnxt;
        nxt = nx2;
        hal = hal2;
        c_xh = n_xh;
        c_T = n_T;
        c_nh = n_nh;
    }

    // block reduction of the partial sums (fixed order, FP64)
    double v[NRED];
    v[R_XHI] = acc_xhi;
    v[R_NHXHI] = acc_nhxhi;
    v[R_NH] = 0.0;  // static: summed once at rt_init
    v[R_N] = acc_N;
    v[R_ABS] = acc_abs * A.vol;
    v[R_ESC] = acc_esc * A.esc_scale;
    v[R_FLOOR] = acc_floor * A.vol;
    v[R_NONFINITE] = double(n_bad);
    v[R_FP64] = double(n_fp64);
    v[R_FALLBACK] = double(n_fb);
#pragma unroll
    for (int hb = 0; hb < 8; ++hb) v[R_HIST0 + hb] = 0.0;
#pragma unroll
    for (int j = 0; j < R_HIST0; ++j) {
        double s = v[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        v[j] = s;
    }
    const int wave = tid >> 6;
    if (lx == 0) {
#pragma unroll
        for (int j = 0; j < R_HIST0; ++j) sred[wave][j] = v[j];
    }
    __syncthreads();
    if (tid < NRED) {
        double s = 0.0;
        if (tid < R_HIST0) {
#pragma unroll
            for (int w = 0; w < NTHREADS / 64; ++w) s += sred[w][tid];
        } else {
            s = double(shist[tid - R_HIST0]);
        }
        A.partials[size_t(blockIdx.x) * NRED + tid] = s;
    }
}

// ---------------------------------------------- finalisation (one block)
// mode 0: a step -- ACC_CUR = sums, ACC_CUM += sums.
// mode 1: initial state -- ACC_CUR = sums, ACC_CUM = 0.
__global__ __launch_bounds__(256) void finalize_kernel(const double *__restrict__ part,
                                                       int nb, double *__restrict__ acc,
                                                       int mode)
{
    __shared__ double s[256];
    const int t = threadIdx.x;
    for (int j = 0; j < NRED; ++j) {
        double v = 0.0;
        for (int b = t; b < nb; b += 256) v += part[size_t(b) * NRED + j];
        s[t] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w) s[t] += s[t + w];
            __syncthreads();
        }
        if (t == 0) {
            acc[ACC_CUR + j] = s[0];
            if (mode == 0)
                acc[ACC_CUM + j] += s[0];
            else
                acc[ACC_CUM + j] = 0.0;
        }
        __syncthreads();
    }
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
    for (uint32_t i = blockIdx.x * 256u + t; i < ncell; i += gridDim.x * 256u) {
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
    const dim3 g(a.nblocks), b(NTHREADS);
    if (a.surr) {
        if (a.mixed)
            hipLaunchKernelGGL((m1_step_kernel<true, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((m1_step_kernel<false, true>), g, b, 0, s, a);
    } else {
        if (a.mixed)
            hipLaunchKernelGGL((m1_step_kernel<true, false>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((m1_step_kernel<false, false>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nblocks, double *acc, int mode,
                           hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, acc,
                       mode);
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
