// Second-Born correlation self-energy on the Matsubara grid (paper Sec. 2.3,
// Eq. sigma2ndb, with both interaction lines between points at equal times):
//
//   Sigma_c,ij(tau) = sum_kl V_ik V_jl [sigma G_ij G_kl Gb_lk - G_il Gb_lk G_kj],
//   Gb = G(beta - tau).
//
// Slices q and q' = n_tau-1-q are done together by one kernel. For each i,
//   M^(i) = Gb diag(V_i,:) G,  i.e.  M^(i)_lj = sum_k Gb_lk V_ik G_kj.
// With symmetric slices everything follows from M^(i):
//   exchange   X_ij  = sum_l G_il  V_jl M^(i)_lj   (slice q)
//              X'_il = sum_j Gb_ij V_lj M^(i)_lj   (slice q')
//   direct     T1_il = M^(i)_ll = sum_k V_ik G_kl Gb_lk,  D_ij = sum_l T1_il V_lj
//   Sigma_c[q]_ij = sigma G_ij D_ij - X_ij,  Sigma_c[q']_ij = sigma Gb_ij D_ij - X'_ij.
// The M^(i) products never reach memory: a workgroup owns one slice pair and
// IB values of i (one per wave), streams l-tiles of 16 rows of M^(i) through
// the matrix cores with the operand A[l][k] = Gb_lk V_ik formed while staging,
// and folds each finished tile into X, X', T1 (registers and LDS). G is read
// and Sigma_c written once per slice pair.
//
// Three arithmetic modes: float64 and float32 on the 16x16x4 MFMA shapes, and
// bf16 operands on the 16x16x32 shape with float32 accumulation. The two
// low-precision modes first scale every slice by an exact power of two
// (2^e_q max|G_q| in [1/2, 1)) and unscale the result, so intermediate products
// of small slices stay in range; only the stored float32 result can underflow.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>
#include <type_traits>

#include "common.h"
#include "mfma.h"

namespace negf {
namespace {

enum { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16 = 2 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BT_LD = 32 + 8;             // row stride (bf16) of the transposed bf16 B panel

template <int MODE>
struct Cfg {
    typedef typename std::conditional<MODE == MODE_F64, double, float>::type T;
    static constexpr int BK = MODE == MODE_BF16 ? 32 : 16;     // k-panel
};

// Per-slice data of the two low-precision modes: ex[q], the power of two every
// slice is scaled by, and for bf16 the scaled slices themselves as bf16, rows
// padded with zeros to ldb (a multiple of 8) elements so that a row is read in
// 16-byte pieces. Since every slice is symmetric, row j of a slice is also the
// k-run of column j that the B operand needs.
struct LowP {
    const int* ex;
    const __bf16* gh;
    int ldb;
};

template <int MODE, int JB>
constexpr size_t stage_bytes() {
    typedef typename Cfg<MODE>::T T;
    // One staging buffer: a B panel [BK][JB*16+1] of T (f64/f32) or [JB*16][BT_LD]
    // of bf16; buffer 0 also holds a [16][JB*16+1] tile of V in T.
    size_t b = MODE == MODE_BF16 ? sizeof(__bf16) * JB * 16 * BT_LD
                                 : sizeof(T) * Cfg<MODE>::BK * (JB * 16 + 1);
    size_t v = sizeof(T) * 16 * (JB * 16 + 1);
    return ((b > v ? b : v) + 15) & ~size_t(15);
}

template <int MODE, int IB, int JB, bool DB, int IPW>
constexpr size_t lds_bytes(int np) {
    typedef typename Cfg<MODE>::T T;
    constexpr int BK = Cfg<MODE>::BK;
    constexpr int IR = IB * IPW;
    const int npj = (np + JB * 16 - 1) / (JB * 16) * (JB * 16);
    return (DB ? 2 : 1) * stage_bytes<MODE, JB>() +
           sizeof(T) * (2 * 16 * (BK + 1) + 2 * IR * BK + (size_t)IR * (3 * np + npj));
}

// Workgroups are handed to the 8 XCDs round-robin by block index; renumber them
// so that each XCD receives a contiguous range of logical blocks (and with it
// all i-blocks of the same slice pair, which then share that XCD's L2).
__device__ __forceinline__ long xcd_remap(long b, long nb) {
    const long x = b & 7, k = b >> 3;
    const long base = nb >> 3, rem = nb & 7;
    return x * base + (x < rem ? x : rem) + k;
}

// Global-to-LDS copy of COUNT elements by NT threads with all of a thread's
// loads in flight before the first store (a strided copy loop waits out one
// memory latency per element). ld(e) returns element e, bounds included;
// st(e, v) writes it.
template <class T, int COUNT, int NT, class Ld, class St>
__device__ __forceinline__ void copy_all(int tid, Ld ld, St st) {
    constexpr int R = (COUNT + NT - 1) / NT;
    T v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = tid + NT * r;
        v[r] = (COUNT % NT == 0 || e < COUNT) ? ld(e) : T(0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = tid + NT * r;
        if (COUNT % NT == 0 || e < COUNT) st(e, v[r]);
    }
}

// minimum waves per SIMD the register allocation must allow for a configuration
template <int MODE, int IB, int JB, bool DB, int IPW>
constexpr int waves_per_eu() {
    // the highest occupancy at which a configuration spills few or no
    // registers (the float64 double-buffered 208-column tile and some float32
    // tiles at four waves per SIMD still spill a little)
    if (IPW > 1) return JB > 4 ? 2 : 3;
    if (MODE == MODE_F64) return JB > 8 ? (IB == 4 ? 1 : 2) : 2;
    if (MODE == MODE_BF16) return JB > 8 ? (IB == 4 ? 1 : 2) : (DB ? 2 : (IB == 4 ? 2 : 4));
    return JB > 8 ? (IB == 4 && DB ? 1 : 2) : (DB ? 3 : 4);
}

// The k-panels of G (B operand), Gb (A operand rows) and V_i (A operand scale)
// are staged through LDS. With DB they are double-buffered: while the matrix
// cores work on panel p, the loads of panel p+1 are in flight into registers,
// then written to the other LDS buffer (one barrier per panel). Without DB a
// panel is loaded, stored and multiplied in turn (two barriers per panel).
// Inside a panel the operand fragments of k-step s+1 are read from LDS while
// the matrix cores work on step s. In bf16 the B panel is copied from the bf16
// slices in 16-byte pieces.
// IPW values of i per wave (IB * IPW per workgroup): with IPW = 2 every B
// fragment read from LDS feeds two matrix-core operations, which halves the
// LDS traffic per flop where that traffic, not the matrix cores, is the limit.
template <int MODE, int IB, int JB, bool DB, int IPW>
__device__ __forceinline__ void s2b_tile(int n, int n_tau, int pair, int iblk, typename Cfg<MODE>::T sigma,
                                         const typename Cfg<MODE>::T* __restrict__ V,
                                         const typename Cfg<MODE>::T* __restrict__ G, LowP lp,
                                         typename Cfg<MODE>::T* __restrict__ Sc, unsigned char* smem_raw) {
    typedef typename Cfg<MODE>::T T;
    constexpr int BK = Cfg<MODE>::BK;
    constexpr int NT = IB * 64;
    constexpr int IR = IB * IPW;                 // rows i per workgroup
    constexpr int GS_LD = JB * 16 + 1;
    // B-panel staging: thread t owns column t % CW of the chunk and rows
    // t / CW + RP r of the panel (r < NSLOT)
    constexpr int CW = JB * 16 <= 64 ? 64 : (JB * 16 <= 128 ? 128 : 256);
    constexpr int RP = NT / CW;
    constexpr int NSLOT = (BK + RP - 1) / RP;
    static_assert(NT % CW == 0, "threads must cover whole staging rows");
    constexpr size_t SB = stage_bytes<MODE, JB>();
    unsigned char* stage0 = smem_raw;
    T* Abuf = reinterpret_cast<T*>(smem_raw + (DB ? 2 : 1) * SB);         // [2][16][BK + 1]
    T* Vbuf = Abuf + 2 * 16 * (BK + 1);                                   // [2][IR][BK]
    const int np = (n + 15) & ~15;
    const int npj = (np + JB * 16 - 1) / (JB * 16) * (JB * 16);          // np padded to whole chunks
    T* T1s = Vbuf + 2 * IR * BK;                                          // [IR][np]  diag of M^(i)
    T* Xs = T1s + IR * np;                                                // [IR][np]  X  (slice q)
    T* XPs = Xs + IR * np;                                                // [IR][np]  X' (slice q')
    T* Gbi = XPs + IR * np;                                               // [IR][npj] row i of Gb (scaled)
    T* Vt = reinterpret_cast<T*>(stage0);                                 // V tile [16][GS_LD] (buffer 0)

    // opaque copy of the thread index: in the persistent kernel this keeps the
    // index arithmetic inside the item loop instead of holding it in registers
    int tid_ = threadIdx.x;
    asm volatile("" : "+v"(tid_));
    const int tid = tid_, lane = tid & 63, w = tid >> 6;
    const int q = pair, qb = n_tau - 1 - pair;
    const bool middle = (q == qb);
    const long nn = (long)n * n;
    const T* Gq = G + (long)q * nn;
    const T* Gb = G + (long)qb * nn;
    T* Sq = Sc + (long)q * nn;
    T* Sqb = Sc + (long)qb * nn;
    // this wave's rows: r = w * IPW + p, i = iblk * IR + r
    const int lc = lane & 15, lg = lane >> 4;
    T sq = T(1), sqb = T(1), uq = T(1), uqb = T(1);
    if constexpr (MODE != MODE_F64) {
        const int* ex = lp.ex;
        sq = (T)ldexpf(1.0f, ex[q]);
        sqb = (T)ldexpf(1.0f, ex[qb]);
        uq = (T)ldexpf(1.0f, -(2 * ex[q] + ex[qb]));
        uqb = (T)ldexpf(1.0f, -(ex[q] + 2 * ex[qb]));
    }
    // bf16: the B panel comes from the bf16 copy of slice q, 16 bytes (8 values
    // of k for one column j) per load
    const __bf16* Ghq = MODE == MODE_BF16 ? lp.gh + (long)q * n * lp.ldb : nullptr;
    constexpr int NV = JB * 16 * (BK / 8);                    // 16-byte pieces per B panel
    constexpr int RBV = (NV + NT - 1) / NT;

    for (int e = tid; e < 3 * IR * np; e += NT) T1s[e] = T(0);     // T1s, Xs, XPs
    for (int e = tid; e < IR * npj; e += NT) {
        const int rr = e / npj, j = e - rr * npj;
        const int ii = iblk * IR + rr;
        Gbi[e] = (ii < n && j < n) ? Gb[(long)ii * n + j] * sqb : T(0);
    }
    // A-operand staging: element tid + NT r of the [16][BK] panel, r < RA
    constexpr int RA = (16 * BK + NT - 1) / NT;
    // V_i staging: element tid + NT r of the [IR][BK] panel, r < RV
    constexpr int RV = (IR * BK + NT - 1) / NT;

    for (int j0 = 0; j0 < np; j0 += JB * 16) {
        const int njb = min(JB, (np - j0) >> 4);
        const int jw = njb * 16;
        const int s_jj = tid % CW, s_kk = tid / CW;
        const bool s_col = s_jj < jw && j0 + s_jj < n;
        // per-lane partial sums of X_ij over the l-tiles, in registers where
        // they fit beside the accumulators; otherwise every l-tile's partial is
        // reduced over the lane groups at once and added into Xs
        constexpr bool XREG = sizeof(T) * JB * IPW <= 56;
        T xcol[IPW][JB];
#pragma unroll
        for (int p = 0; p < IPW; ++p)
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) xcol[p][jb] = T(0);

        constexpr int NJB = JB;   // the last chunk is padded with zero columns
#pragma unroll 1
        for (int l0 = 0; l0 < n; l0 += 16) {
            typename Mma<T>::acc_t acc[IPW][NJB];
#pragma unroll
            for (int p = 0; p < IPW; ++p)
#pragma unroll
                for (int jb = 0; jb < NJB; ++jb) acc[p][jb] = Mma<T>::zero();
            T rg[MODE == MODE_BF16 ? 1 : NSLOT], ra[RA], rv[RV];
            uint4 rgv[MODE == MODE_BF16 ? RBV : 1];
            auto load = [&](int k0) {
                if constexpr (MODE == MODE_BF16) {
#pragma unroll
                    for (int r = 0; r < RBV; ++r) {
                        const int v = tid + NT * r, jj = v / (BK / 8), k = k0 + 8 * (v % (BK / 8));
                        const int j = j0 + jj;
                        rgv[r] = (v < NV && jj < jw && j < n && k < lp.ldb)
                                     ? *reinterpret_cast<const uint4*>(Ghq + (long)j * lp.ldb + k)
                                     : uint4{0u, 0u, 0u, 0u};
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < NSLOT; ++r) {
                        const int kk = s_kk + RP * r, k = k0 + kk;
                        rg[r] = (s_col && kk < BK && k < n) ? Gq[(long)k * n + j0 + s_jj] : T(0);
                    }
                }
#pragma unroll
                for (int r = 0; r < RA; ++r) {
                    const int e = tid + NT * r, ll = e / BK, kk = e - ll * BK;
                    const int l = l0 + ll, k = k0 + kk;
                    ra[r] = (e < 16 * BK && l < n && k < n) ? Gb[(long)l * n + k] : T(0);
                }
#pragma unroll
                for (int r = 0; r < RV; ++r) {
                    const int e = tid + NT * r, rr = e / BK, kk = e - rr * BK;
                    const int vi = iblk * IR + rr, k = k0 + kk;
                    rv[r] = (e < IR * BK && vi < n && k < n) ? V[(long)vi * n + k] : T(0);
                }
            };
            auto store = [&](int buf) {
                unsigned char* sb = stage0 + buf * SB;
                if constexpr (MODE == MODE_BF16) {
#pragma unroll
                    for (int r = 0; r < RBV; ++r) {
                        const int v = tid + NT * r, jj = v / (BK / 8), g = v % (BK / 8);
                        if (v < NV) *reinterpret_cast<uint4*>(reinterpret_cast<__bf16*>(sb) + jj * BT_LD + 8 * g) = rgv[r];
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < NSLOT; ++r) {
                        const int kk = s_kk + RP * r;
                        if (s_jj < JB * 16 && kk < BK) reinterpret_cast<T*>(sb)[kk * GS_LD + s_jj] = rg[r] * sq;
                    }
                }
#pragma unroll
                for (int r = 0; r < RA; ++r) {
                    const int e = tid + NT * r, ll = e / BK, kk = e - ll * BK;
                    if (e < 16 * BK) Abuf[buf * 16 * (BK + 1) + ll * (BK + 1) + kk] = ra[r] * sqb;
                }
#pragma unroll
                for (int r = 0; r < RV; ++r) {
                    const int e = tid + NT * r;
                    if (e < IR * BK) Vbuf[buf * IR * BK + e] = rv[r];
                }
            };
            const int npan = (n + BK - 1) / BK;
            if constexpr (DB) {
                load(0);
                __syncthreads();                  // previous readers of buffer 0 (V tile) are done
                store(0);
                __syncthreads();
            }
#pragma unroll 1
            for (int pn = 0; pn < npan; ++pn) {
                const int buf = DB ? (pn & 1) : 0;
                const bool more = DB && pn + 1 < npan;
                if constexpr (!DB) {
                    load(pn * BK);
                    __syncthreads();
                    store(0);
                    __syncthreads();
                }
                if (more) load((pn + 1) * BK);
                const T* Ab = Abuf + buf * 16 * (BK + 1);
                const T* Vk = Vbuf + buf * IR * BK;
                if constexpr (MODE == MODE_BF16) {
                    const __bf16* Bt = reinterpret_cast<const __bf16*>(stage0 + buf * SB);
                    bf16x8 a[IPW];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int kk = lg * 8 + e;
                        const T av = Ab[lc * (BK + 1) + kk];
#pragma unroll
                        for (int p = 0; p < IPW; ++p) a[p][e] = (__bf16)(float)(av * Vk[(w * IPW + p) * BK + kk]);
                    }
#pragma unroll
                    for (int jb = 0; jb < NJB; ++jb) {
                        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bt[(jb * 16 + lc) * BT_LD + lg * 8]);
#pragma unroll
                        for (int p = 0; p < IPW; ++p)
                            acc[p][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[p], b, acc[p][jb], 0, 0, 0);
                    }
                } else {
                    const T* Gs = reinterpret_cast<const T*>(stage0 + buf * SB);
                    // k-steps of 4 that hold real rows (uniform across the workgroup)
                    const int nks = min(BK / 4, (n - pn * BK + 3) >> 2);
                    // float64 runs on the four-block 4x4x4 shape, which sustains
                    // about 1.5x the rate of the 16x16x4 one on gfx950: four of
                    // them (rows 4r .. 4r+3 of the l-tile) make one 16 x 16 tile.
                    // With the same A rows in all four blocks, block b holds
                    // columns 4b .. 4b+3, so B and the result use the lanes and
                    // registers of the 16x16x4 shape (row 4r + lane/16, column
                    // lane % 16); A row 4r + lane % 4, k = lane / 16.
                    constexpr bool QUAD = MODE == MODE_F64;
                    constexpr int NA = QUAD ? 4 : 1;
                    // row groups of 4 that hold real rows (uniform): the padded
                    // groups of the last l-tile are skipped
                    const int nrg = QUAD ? min(4, (n - l0 + 3) >> 2) : 1;
                    // operand fragments in two register sets: the LDS reads of
                    // k-step ks + 1 are in flight while the matrix cores work on ks
                    T fa[2][NA], fv[2][IPW], fb[2][NJB];
                    auto frag = [&](int ks, int s) {
                        const int kk = ks * 4 + lg;
                        if constexpr (QUAD) {
#pragma unroll
                            for (int r = 0; r < NA; ++r) fa[s][r] = Ab[(4 * r + (lane & 3)) * (BK + 1) + kk];
                        } else {
                            fa[s][0] = Ab[lc * (BK + 1) + kk];
                        }
#pragma unroll
                        for (int p = 0; p < IPW; ++p) fv[s][p] = Vk[(w * IPW + p) * BK + kk];
#pragma unroll
                        for (int jb = 0; jb < NJB; ++jb) fb[s][jb] = Gs[kk * GS_LD + jb * 16 + lc];
                    };
                    frag(0, 0);
#pragma unroll
                    for (int ks = 0; ks < BK / 4; ++ks) {
                        if (ks < nks) {
                            const int s = ks & 1;
                            if (ks + 1 < nks) frag(ks + 1, s ^ 1);
                            if constexpr (QUAD) {
#pragma unroll
                                for (int r = 0; r < NA; ++r) {
                                    if (r < nrg) {
#pragma unroll
                                        for (int p = 0; p < IPW; ++p) {
                                            const double a = fa[s][r] * fv[s][p];
#pragma unroll
                                            for (int jb = 0; jb < NJB; ++jb)
                                                acc[p][jb][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                                                    a, fb[s][jb], acc[p][jb][r], 0, 0, 0);
                                        }
                                    }
                                }
                            } else {
                                T a[IPW];
#pragma unroll
                                for (int p = 0; p < IPW; ++p) a[p] = fa[s][0] * fv[s][p];
#pragma unroll
                                for (int jb = 0; jb < NJB; ++jb)
#pragma unroll
                                    for (int p = 0; p < IPW; ++p)
                                        acc[p][jb] = Mma<T>::mma(a[p], fb[s][jb], acc[p][jb]);
                            }
                        }
                    }
                }
                if constexpr (DB) {
                    if (more) store(buf ^ 1);
                    __syncthreads();
                }
            }
            if constexpr (!DB) __syncthreads();
            // diagonal of M^(i) for rows l0..l0+15 if this chunk holds those columns
            if (l0 >= j0 && l0 < j0 + jw) {
                const int jd = (l0 - j0) >> 4;
#pragma unroll
                for (int jb = 0; jb < NJB; ++jb)
                    if (jb == jd) {
#pragma unroll
                        for (int p = 0; p < IPW; ++p)
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                if (Mma<T>::row(lane, r) == lc) T1s[(w * IPW + p) * np + l0 + lc] = acc[p][jb][r];
                    }
            }
            // V rows l0..l0+15 (this chunk's columns, zero-padded) into buffer 0;
            // float32 storage has the registers to keep all of a thread's loads
            // in flight (float64 copies element by element: its accumulators
            // leave no room)
            {
                auto ld = [&](int e) {
                    const int ll = e / (JB * 16), jj = e - ll * (JB * 16);
                    const int l = l0 + ll, j = j0 + jj;
                    return (l < n && jj < jw && j < n) ? V[(long)l * n + j] : T(0);
                };
                auto st = [&](int e, T v) {
                    const int ll = e / (JB * 16), jj = e - ll * (JB * 16);
                    Vt[ll * GS_LD + jj] = v;
                };
                if constexpr (MODE == MODE_F64) {
                    for (int e = tid; e < 16 * JB * 16; e += NT) st(e, ld(e));
                } else {
                    copy_all<T, 16 * JB * 16, NT>(tid, ld, st);
                }
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < IPW; ++p) {
                const int rr = w * IPW + p, i = iblk * IR + rr;
                const bool iok = i < n;
                T gil[4], xp[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int l = l0 + Mma<T>::row(lane, r);
                    gil[r] = (iok && l < n) ? Gq[(long)i * n + l] * sq : T(0);
                    xp[r] = T(0);
                }
#pragma unroll
                for (int jb = 0; jb < NJB; ++jb) {
                    T xc = T(0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const T vm = Vt[Mma<T>::row(lane, r) * GS_LD + jb * 16 + lc] * acc[p][jb][r];
                        xp[r] += Gbi[rr * npj + j0 + jb * 16 + lc] * vm;
                        xc += gil[r] * vm;
                    }
                    if constexpr (XREG) {
                        xcol[p][jb] += xc;
                    } else {
                        const T sx = sum4x16(xc);
                        if (jb < njb && lg == 0) Xs[rr * np + j0 + jb * 16 + lc] += sx;
                    }
                }
                // X'_il (slice q'), partial over this chunk's columns
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const T sx = sum16(xp[r]);
                    const int l = l0 + Mma<T>::row(lane, r);
                    if (lc == 0) XPs[rr * np + l] += sx;
                }
            }
        }
        // X_ij (slice q) for this chunk's columns
        if constexpr (XREG) {
#pragma unroll
            for (int p = 0; p < IPW; ++p)
#pragma unroll
                for (int jb = 0; jb < JB; ++jb) {
                    const T sx = sum4x16(xcol[p][jb]);
                    if (jb < njb && lg == 0) Xs[(w * IPW + p) * np + j0 + jb * 16 + lc] = sx;
                }
        }
    }

    // direct term D_ij = sum_l T1_il V_lj, then one store per output element
    constexpr int DM = (JB * 16 + 63) / 64;
    for (int j0 = 0; j0 < np; j0 += JB * 16) {
        const int jw = min(JB * 16, np - j0);
        T d[IPW][DM];
#pragma unroll
        for (int p = 0; p < IPW; ++p)
#pragma unroll
            for (int m = 0; m < DM; ++m) d[p][m] = T(0);
        for (int l0 = 0; l0 < n; l0 += 16) {
            if constexpr (MODE == MODE_F64) {
                __syncthreads();
                for (int e = tid; e < 16 * jw; e += NT) {
                    const int ll = e / jw, jj = e - ll * jw;
                    const int l = l0 + ll, j = j0 + jj;
                    Vt[ll * GS_LD + jj] = (l < n && j < n) ? V[(long)l * n + j] : T(0);
                }
            } else {
                // all loads in flight, then the barrier that lets the stores
                // replace the tile the previous l-step read
                constexpr int R = (16 * JB * 16 + NT - 1) / NT;
                T v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int e = tid + NT * r, ll = e / (JB * 16), jj = e - ll * (JB * 16);
                    const int l = l0 + ll, j = j0 + jj;
                    v[r] = (e < 16 * JB * 16 && l < n && jj < jw && j < n) ? V[(long)l * n + j] : T(0);
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int e = tid + NT * r, ll = e / (JB * 16), jj = e - ll * (JB * 16);
                    if (e < 16 * JB * 16) Vt[ll * GS_LD + jj] = v[r];
                }
            }
            __syncthreads();
            for (int ll = 0; ll < 16; ++ll) {
#pragma unroll
                for (int p = 0; p < IPW; ++p) {
                    const T t = (l0 + ll < n) ? T1s[(w * IPW + p) * np + l0 + ll] : T(0);
#pragma unroll
                    for (int m = 0; m < DM; ++m)
                        if (lane + 64 * m < jw) d[p][m] += t * Vt[ll * GS_LD + lane + 64 * m];
                }
            }
        }
#pragma unroll
        for (int p = 0; p < IPW; ++p) {
            const int rr = w * IPW + p, i = iblk * IR + rr;
            if (i < n) {
#pragma unroll
                for (int m = 0; m < DM; ++m) {
                    const int j = j0 + lane + 64 * m;
                    if (lane + 64 * m < jw && j < n) {
                        const long ij = (long)i * n + j;
                        Sq[ij] = (sigma * (Gq[ij] * sq) * d[p][m] - Xs[rr * np + j]) * uq;
                        if (!middle) Sqb[ij] = (sigma * (Gb[ij] * sqb) * d[p][m] - XPs[rr * np + j]) * uqb;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- float64, direct-to-LDS staging
// The float64 tile with the same arithmetic as s2b_tile (four-block 4x4x4
// MFMAs, same epilogue and direct term), but every operand panel reaches LDS
// by direct global->LDS loads (global_load_lds_dwordx4: each lane moves 16
// bytes, the wave's 64 pieces land contiguously at the address in M0), so no
// register holds staged data. The k-panels are double-buffered: the loads of
// panel p+1 are in flight while the matrix cores work on panel p, with one
// barrier per panel. The loads read zero-padded copies of G and V (rows and
// columns padded to np = n rounded up to 16), so every piece is in bounds and
// the padding is exact zeros.
namespace dma {

// A panel [16 l][BK k]. With BK = 16 the 16-byte piece kp (k = 2 kp, 2 kp + 1)
// of row l is stored at piece kp ^ (l & 7) of that row, so the fragment reads
// of four rows 128 bytes apart spread over the banks; with BK = 4 the four rows
// a fragment read touches are 32 bytes apart and the layout is plain.
template <int BK>
__device__ __forceinline__ int a_index(int l, int k) {
    if constexpr (BK == 16) return l * 16 + ((((k >> 1) ^ (l & 7))) << 1) + (k & 1);
    else return l * BK + k;
}

template <int IB, int JB, int BK>
struct Layout {
    static_assert(BK == 16 || BK == 4, "k-panel of 16 or 4");
    static constexpr int JW = JB * 16;
    static constexpr int B_EL = BK * JW;             // B panel [BK][jw] (row stride jw of the chunk)
    static constexpr int A_EL = 16 * BK;
    static constexpr int V_EL = IB * BK;             // V panel [IB][BK]
    static constexpr int STAGE_EL = B_EL + A_EL + V_EL;
    static constexpr int VT_EL = 16 * JW + IB * 16;  // V tile of the epilogue [16][jw], then G_il [IB][16]
    // one column chunk: the direct term is accumulated in the l-tile loop,
    // in a further [IB][np] array
    static size_t bytes(int np) {
        const int npj = (np + JW - 1) / JW * JW;
        const size_t d = np <= JW ? (size_t)IB * np : 0;
        return sizeof(double) * (2 * (size_t)STAGE_EL + VT_EL + 3 * (size_t)IB * np + (size_t)IB * npj + d);
    }
};

__device__ __forceinline__ void load16(const double* g, double* lds_wave) {
    __builtin_amdgcn_global_load_lds(static_cast<const void*>(g), (__attribute__((address_space(3))) void*)lds_wave,
                                     16, 0, 0);
}
// The same from a wave-uniform base and a 32-bit per-lane byte offset, which
// the instruction takes as a scalar base plus one vector register: the offsets
// of a chunk then stay in one register each through the panel loop.
__device__ __forceinline__ void load16(const double* base, unsigned byte_off, double* lds_wave) {
    load16(reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + byte_off), lds_wave);
}

// Pieces 0 .. count-1 of a contiguous LDS region, piece c from src(c); the
// waves take 64 consecutive pieces each in turn.
template <int NT, class F>
__device__ __forceinline__ void copy(double* dst, int count, int tid, F src) {
    const int w = tid >> 6, lane = tid & 63;
    for (int base = w * 64; base < count; base += NT) {
        const int c = base + lane;
        if (c < count) load16(src(c), dst + 2 * base);
    }
}

__device__ __forceinline__ void wait_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <int IB, int JB, int BK>
__device__ __forceinline__ void tile(int n, int np, int n_tau, int pair, int iblk, double sigma,
                                     const double* __restrict__ Vp, const double* __restrict__ Gp,
                                     const double* __restrict__ G, double* __restrict__ Sc, double* smem, int lbeg,
                                     int lend, double* __restrict__ pd, double* __restrict__ px) {
    typedef Layout<IB, JB, BK> L;
    constexpr int NT = IB * 64;
    constexpr int JW = L::JW;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lc = lane & 15, lg = lane >> 4;
    const int q = pair, qb = n_tau - 1 - pair;
    const bool middle = q == qb;
    const long nn = (long)n * n, pp = (long)np * np;
    const double* Gq = Gp + (long)q * pp;            // padded slices
    const double* Gb = Gp + (long)qb * pp;
    const int npj = (np + JW - 1) / JW * JW;
    double* stage = smem;                            // [2][STAGE_EL]
    double* Vt = stage + 2 * L::STAGE_EL;            // [16][jw]
    double* Gil = Vt + 16 * JW;                      // [IB][16]
    double* T1s = Vt + L::VT_EL;                     // [IB][np]
    double* Xs = T1s + IB * np;                      // [IB][np]
    double* XPs = Xs + IB * np;                      // [IB][np]
    double* Gbi = XPs + IB * np;                     // [IB][npj]
    double* Ds = Gbi + IB * npj;                     // [IB][np], one column chunk only
    const bool one_chunk = np <= JW;
    const int i = iblk * IB + w;                     // this wave's row (< np)

    for (int e = tid; e < 3 * IB * np; e += NT) T1s[e] = 0.0;
    if (one_chunk)
        for (int e = tid; e < IB * np; e += NT) Ds[e] = 0.0;
    for (int e = tid; e < IB * npj; e += NT) {
        const int rr = e / npj, j = e - rr * npj;
        Gbi[e] = j < np ? Gb[(long)(iblk * IB + rr) * np + j] : 0.0;
    }
    const int npan = (n + BK - 1) / BK;

    for (int j0 = 0; j0 < np; j0 += JW) {
        const int jw = min(JW, np - j0);
        const int njb = jw >> 4;
        // Element offsets of this lane's 16-byte pieces, the same for every panel
        // of the chunk: piece c of a [rows][jw] block (B panel: BK rows, V tile:
        // 16 rows) is row c / (jw/2), columns 2 (c % (jw/2)) + 0, 1; the waves
        // take 64 consecutive pieces each in turn. A and V pieces as in the
        // panel layouts.
        constexpr int NPV = (16 * (JW / 2) + NT - 1) / NT;      // V-tile pieces per lane
        constexpr int NPB = (BK * (JW / 2) + NT - 1) / NT;      // B-panel pieces per lane
        // (byte offsets; ~0u marks a piece that does not exist)
        constexpr unsigned kNone = ~0u;
        const int hp = jw >> 1;
        unsigned offb[NPV];
#pragma unroll
        for (int t = 0; t < NPV; ++t) {
            const int c = w * 64 + t * NT + lane;
            const int kk = c / hp, jp = c - kk * hp;
            offb[t] = c < 16 * hp ? 8u * (unsigned)(kk * np + j0 + 2 * jp) : kNone;
        }
        // A pieces (16 rows of BK/2): the last waves; V pieces (IB rows of BK/2):
        // the wave before them
        constexpr int NA = 16 * BK / 2, AW = (NA + 63) / 64;
        const int ca = tid - (NT - 64 * AW);
        const int ra = ca / (BK / 2), pa = ca % (BK / 2);
        const unsigned offa =
            (ca >= 0 && ca < NA) ? 8u * (unsigned)(ra * np + 2 * (BK == 16 ? (pa ^ (ra & 7)) : pa)) : kNone;
        const int cg = tid - 128;                    // G_il pieces of the epilogue: the third wave
        const int cv = tid - (NT - 64 * AW - 64);
        const unsigned offv = (cv >= 0 && cv < IB * BK / 2)
                                  ? 8u * (unsigned)((iblk * IB + cv / (BK / 2)) * np + 2 * (cv % (BK / 2)))
                                  : kNone;
        // all pieces of the [rows][jw] block of M (row stride np) that starts
        // row0 rows down, into dst. The row offset is added to the 32-bit piece
        // offsets (one slice is far below 4 GiB) and the base stays the slice
        // pointer, so no 64-bit address is kept per piece across panels.
        auto copy_rows = [&](double* dst, const double* M, int row0, auto rows_t) {
            constexpr int ROWS = decltype(rows_t)::value;
            constexpr int NP = ROWS == 16 ? NPV : NPB;
            const unsigned ro = 8u * (unsigned)(row0 * np);
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                const bool ok = ROWS == 16 ? offb[t] != kNone : (w * 64 + t * NT + lane < ROWS * hp);
                if (ok) load16(M, offb[t] + ro, dst + 2 * (w * 64 + t * NT));
            }
        };
        auto issue = [&](int l0, int pn, int buf) {
            double* sb = stage + buf * L::STAGE_EL;
            const int k0 = pn * BK;
            copy_rows(sb, Gq, k0, std::integral_constant<int, BK>());
            if (offa != kNone) load16(Gb, offa + 8u * (unsigned)(l0 * np + k0), sb + L::B_EL + 2 * (ca & ~63));
            if (offv != kNone) load16(Vp, offv + 8u * (unsigned)k0, sb + L::B_EL + L::A_EL + 2 * (cv & ~63));
        };
        int g = 0;                                   // panels started in this chunk
        issue(lbeg, 0, 0);
        wait_loads();
        __syncthreads();
        for (int l0 = lbeg; l0 < lend; l0 += 16) {
            // V rows l0 .. l0+15 of this chunk for the epilogue; G_il for this wave's rows
            copy_rows(Vt, Vp, l0, std::integral_constant<int, 16>());
            if (cg >= 0 && cg < IB * 8) load16(Gq, 8u * (unsigned)((iblk * IB + (cg >> 3)) * np + l0 + 2 * (cg & 7)), Gil);
            dv4 acc[JB];
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) acc[jb] = Mma<double>::zero();
            const int nrg = min(4, (n - l0 + 3) >> 2);   // groups of 4 rows l holding l < n
#pragma unroll 1
            for (int pn = 0; pn < npan; ++pn, ++g) {
                const int cur = g & 1;
                if (pn + 1 < npan) issue(l0, pn + 1, cur ^ 1);
                else if (l0 + 16 < lend) issue(l0 + 16, 0, cur ^ 1);
                const double* Bs = stage + cur * L::STAGE_EL;
                const double* As = Bs + L::B_EL;
                const double* Vs = As + L::A_EL;
                // A branch-free body: the padding rows and columns of the copies
                // are zeros, so the ragged last panel and l-tile are computed
                // whole, and in a narrow last chunk the column blocks past jw read
                // other staged values (finite; their results are never used).
                // The operand reads of k-step ks + 1 are issued before the products
                // of ks.
                double fa[2][4], fv[2], fb[2][JB];
                auto frag = [&](int ks, int s) {
                    const int kk = ks * 4 + lg;
#pragma unroll
                    for (int r = 0; r < 4; ++r) fa[s][r] = As[a_index<BK>(4 * r + (lane & 3), kk)];
                    fv[s] = Vs[w * BK + kk];
#pragma unroll
                    for (int jb = 0; jb < JB; ++jb) fb[s][jb] = Bs[kk * jw + jb * 16 + lc];
                };
                // k-steps of the last panel past k = n and row groups of the
                // last l-tile past l = n hold zero padding only: skipped
                // (uniform branches; the results are the same)
                const int nks = min(BK / 4, (n - pn * BK + 3) >> 2);
                frag(0, 0);
#pragma unroll
                for (int ks = 0; ks < BK / 4; ++ks) {
                    const int s = ks & 1;
                    if (ks + 1 < BK / 4) frag(ks + 1, s ^ 1);
                    if (ks == 0 || ks < nks) {
                        double a[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) a[r] = fa[s][r] * fv[s];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (r == 0 || r < nrg)
#pragma unroll
                                for (int jb = 0; jb < JB; ++jb)
                                    acc[jb][r] =
                                        __builtin_amdgcn_mfma_f64_4x4x4f64(a[r], fb[s][jb], acc[jb][r], 0, 0, 0);
                    }
                }
                wait_loads();
                __syncthreads();
            }
            // diagonal of M^(i) for rows l0 .. l0+15 if this chunk holds those columns
            if (l0 >= j0 && l0 < j0 + jw) {
                const int jd = (l0 - j0) >> 4;
#pragma unroll
                for (int jb = 0; jb < JB; ++jb)
                    if (jb == jd) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (Mma<double>::row(lane, r) == lc) T1s[w * np + l0 + lc] = acc[jb][r];
                    }
            }
            double xp[4] = {0.0, 0.0, 0.0, 0.0}, gil[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) gil[r] = Gil[w * 16 + Mma<double>::row(lane, r)];
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) {
                if (jb < njb) {
                    const double gbi = Gbi[w * npj + j0 + jb * 16 + lc];
                    double xc = 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double vm = Vt[Mma<double>::row(lane, r) * jw + jb * 16 + lc] * acc[jb][r];
                        xp[r] += gbi * vm;
                        xc += gil[r] * vm;
                    }
                    const double sx = sum4x16(xc);
                    if (lg == 0) Xs[w * np + j0 + jb * 16 + lc] += sx;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double sx = sum16(xp[r]);
                if (lc == 0) XPs[w * np + l0 + Mma<double>::row(lane, r)] += sx;
            }
            if (one_chunk) {
                // direct term D_ij += sum_l T1_il V_lj over this tile's 16 rows l,
                // with the V rows already in Vt (this wave wrote T1 above; its own
                // LDS operations complete in order)
                constexpr int DM = (JW + 63) / 64;
#pragma unroll
                for (int m = 0; m < DM; ++m) {
                    const int j = lane + 64 * m;
                    if (j < jw) {
                        double d = Ds[w * np + j];
#pragma unroll
                        for (int ll = 0; ll < 16; ++ll) d += T1s[w * np + l0 + ll] * Vt[ll * jw + j];
                        Ds[w * np + j] = d;
                    }
                }
            }
            __syncthreads();                         // Vt is read; the next l-tile may replace it
        }
    }

    // The output phase takes its per-lane indices from an opaque copy of the
    // thread index, so that none computed before the loops has to stay live
    // (and spill) through them.
    int tid_o = threadIdx.x;
    asm volatile("" : "+v"(tid_o));
    {
        const int tid = tid_o, lane = tid & 63, w = tid >> 6, i = iblk * IB + w;
        // direct term D_ij = sum_l T1_il V_lj (V tiles double-buffered through the
        // stage area), then one store per output element
        constexpr int DM = (JW + 63) / 64;
        for (int j0 = 0; j0 < np; j0 += JW) {
            const int jw = min(JW, np - j0);
            double d[DM];
#pragma unroll
            for (int m = 0; m < DM; ++m) d[m] = 0.0;
            if (one_chunk) {
#pragma unroll
                for (int m = 0; m < DM; ++m)
                    if (lane + 64 * m < jw) d[m] = Ds[w * np + lane + 64 * m];
            } else {
                // V tiles of DR rows, as many as one stage buffer holds
                constexpr int DR = BK;
                static_assert(DR * JW <= L::STAGE_EL, "a V tile must fit a stage buffer");
                auto issue_v = [&](int l0, int buf) {
                    copy<NT>(stage + buf * L::STAGE_EL, DR * (jw >> 1), tid, [&](int c) {
                        const int hp = jw >> 1, ll = c / hp, jp = c - ll * hp;
                        return Vp + (long)(l0 + ll) * np + j0 + 2 * jp;
                    });
                };
                issue_v(0, 0);
                int b = 0;
                for (int l0 = 0; l0 < n; l0 += DR, b ^= 1) {
                    wait_loads();
                    __syncthreads();
                    if (l0 + DR < n) issue_v(l0 + DR, b ^ 1);
                    const double* Vv = stage + b * L::STAGE_EL;
                    for (int ll = 0; ll < DR; ++ll) {
                        const double t = T1s[w * np + l0 + ll];      // zero beyond n
#pragma unroll
                        for (int m = 0; m < DM; ++m)
                            if (lane + 64 * m < jw) d[m] += t * Vv[ll * jw + lane + 64 * m];
                    }
                }
            }
            if (i < n && px) {
                // one part of the l range: D and X of this part, summed over
                // the parts by k_s2b_parts_sum
#pragma unroll
                for (int m = 0; m < DM; ++m) {
                    const int j = j0 + lane + 64 * m;
                    if (lane + 64 * m < jw && j < n) {
                        pd[(long)i * np + j] = d[m];
                        px[(long)i * np + j] = Xs[w * np + j];
                    }
                }
            } else if (i < n) {
                // G_ij of slice q from the padded copy (its rows were streamed
                // through the L2 by the panels just before), of slice q' from
                // the row already in LDS
                double* Sq = Sc + (long)q * nn;
                double* Sqb = Sc + (long)qb * nn;
#pragma unroll
                for (int m = 0; m < DM; ++m) {
                    const int j = j0 + lane + 64 * m;
                    if (lane + 64 * m < jw && j < n) {
                        const long ij = (long)i * n + j;
                        Sq[ij] = sigma * Gq[(long)i * np + j] * d[m] - Xs[w * np + j];
                        if (!middle) Sqb[ij] = sigma * Gbi[w * npj + j] * d[m] - XPs[w * np + j];
                    }
                }
            }
            __syncthreads();                             // before the next chunk reuses the stage area
        }
    }
}

}  // namespace dma

// Zero-padded copy of a stack of n x n matrices into np x np blocks (np a
// multiple of 16): grid y runs over the matrices, and each thread writes two
// adjacent padded elements with one 16-byte store (32-bit index arithmetic
// within a matrix).
__global__ __launch_bounds__(256) void k_pad_copy(int n, int np, long count, const double* __restrict__ src,
                                                  double* __restrict__ dst) {
    const int hp = np * np / 2;
    for (long s = blockIdx.y; s < count; s += gridDim.y) {
        const double* a = src + s * n * n;
        double2* b = reinterpret_cast<double2*>(dst + s * np * np);
        for (int e = blockIdx.x * 256 + threadIdx.x; e < hp; e += gridDim.x * 256) {
            const int r = 2 * e / np, c = 2 * e - r * np;
            double2 v;
            v.x = (r < n && c < n) ? a[r * n + c] : 0.0;
            v.y = (r < n && c + 1 < n) ? a[r * n + c + 1] : 0.0;
            b[e] = v;
        }
    }
}

// Workgroups below n_full take one (slice pair, i-block) each. With n_parts > 0
// the middle slice (tau = beta/2, paired with itself, the last pair) is left out
// of them: it would be the last round of the launch, with most CUs idle. The
// n_parts x n_iblk workgroups after n_full take it instead, each one part of its
// l-tiles, and write their D and X terms to part (n_parts blocks of
// [D | X], each [n_iblk IB][np]).
template <int IB, int JB, int BK>
__global__ __launch_bounds__(IB * 64, 2) void k_sigma2b_dma(int n, int np, int n_tau, int n_iblk, double sigma,
                                                            const double* __restrict__ Vp,
                                                            const double* __restrict__ Gp,
                                                            const double* __restrict__ G, double* __restrict__ Sc,
                                                            long n_full, int n_parts, double* __restrict__ part) {
    extern __shared__ __align__(16) double smem_d[];
    const long b = blockIdx.x;
    int pair, iblk, lbeg = 0, lend = n;
    double *pd = nullptr, *px = nullptr;
    if (b < n_full) {
        const long lb = xcd_remap(b, n_full);
        pair = (int)(lb / n_iblk);
        iblk = (int)(lb % n_iblk);
    } else {
        const int u = (int)(b - n_full), sp = u / n_iblk;
        const int nlt = (n + 15) >> 4;
        const long ni = (long)n_iblk * IB * np;
        pair = (n_tau - 1) / 2;
        iblk = u - sp * n_iblk;
        lbeg = 16 * (sp * nlt / n_parts);
        lend = min(n, 16 * ((sp + 1) * nlt / n_parts));
        pd = part + 2 * ni * sp;
        px = pd + ni;
    }
    dma::tile<IB, JB, BK>(n, np, n_tau, pair, iblk, sigma, Vp, Gp, G, Sc, smem_d, lbeg, lend, pd, px);
}

// Sigma_c of the middle slice from the parts: sigma G_ij sum D - sum X
__global__ void k_s2b_parts_sum(int n, int np, long ni, int n_parts, double sigma, const double* __restrict__ Gm,
                                const double* __restrict__ part, double* __restrict__ Sm) {
    const long nn = (long)n * n;
    for (long e = blockIdx.x * 256L + threadIdx.x; e < nn; e += (long)gridDim.x * 256) {
        const int i = (int)(e / n), j = (int)(e - (long)i * n);
        const long o = (long)i * np + j;
        double d = 0.0, x = 0.0;
        for (int sp = 0; sp < n_parts; ++sp) {
            d += part[2 * ni * sp + o];
            x += part[2 * ni * sp + ni + o];
        }
        Sm[e] = sigma * Gm[e] * d - x;
    }
}

// ---------------------------------------------------------------- float64 on the vector ALUs
// On gfx950 the float64 vector FMA sustains more than the 16x16x4 float64 matrix
// instruction (measured: ~72 vs ~48 TFLOP/s; the four-block 4x4x4 form reaches
// ~75), so the float64 mode also has tiles that form M^(i) with plain FMAs. A wave still owns one i; its 64 lanes form an 8 x 8
// grid and lane (ty, tx) accumulates a TL x TL block of a HT x HT tile of M^(i)
// (HT = 8 TL), rows l = l0 + ty TL + a, columns j = j0 + tx TL + b. The k-panels
// of Gb (rows l) and G (columns j) are staged in LDS (shared by the IB waves);
// V_i is applied to the Gb values as they are read. The epilogue is the same
// arithmetic as in the matrix-core tile (diagonal, X', X), with the row and
// column sums reduced across the 8 lanes of a lane row or column.
constexpr int VK = 32;   // k-panel of the vector-ALU tiles

template <int IB, int TL, int IPW>
constexpr size_t lds_bytes_valu(int n) {
    constexpr int HT = 8 * TL;
    const int npt = (n + HT - 1) / HT * HT;
    const size_t stage = 2 * VK * HT;
    const size_t vt = (size_t)HT * (HT + 1);
    return sizeof(double) * ((stage > vt ? stage : vt) + (size_t)IB * IPW * VK + 4 * (size_t)IB * IPW * npt);
}

// IPW values of i per wave share every Gb and G value read from LDS.
template <int IB, int TL, int IPW>
__device__ __forceinline__ void s2b_tile_valu(int n, int n_tau, int pair, int iblk, double sigma,
                                              const double* __restrict__ V, const double* __restrict__ G,
                                              double* __restrict__ Sc, unsigned char* smem_raw) {
    constexpr int NT = IB * 64;
    constexpr int IR = IB * IPW;
    constexpr int HT = 8 * TL;
    constexpr int VLD = HT + 1;
    const int npt = (n + HT - 1) / HT * HT;
    double* Ap = reinterpret_cast<double*>(smem_raw);        // [VK][HT]  Gb[l][k] by k
    double* Bp = Ap + VK * HT;                               // [VK][HT]  G[k][j]
    double* Vt = Ap;                                          // [HT][VLD] V tile (epilogue)
    constexpr size_t STG = (2 * VK * HT > HT * VLD) ? 2 * VK * HT : HT * VLD;
    double* Vp = Ap + STG;                                    // [IR][VK]  V_i panel
    double* T1s = Vp + IR * VK;                               // [IR][npt]
    double* Xs = T1s + IR * npt;
    double* XPs = Xs + IR * npt;
    double* Gbi = XPs + IR * npt;                             // [IR][npt] row i of Gb

    int tid_ = threadIdx.x;
    asm volatile("" : "+v"(tid_));
    const int tid = tid_, lane = tid & 63, w = tid >> 6;
    const int tx = lane & 7, ty = lane >> 3;
    const int q = pair, qb = n_tau - 1 - pair;
    const bool middle = (q == qb);
    const long nn = (long)n * n;
    const double* Gq = G + (long)q * nn;
    const double* Gb = G + (long)qb * nn;
    double* Sq = Sc + (long)q * nn;
    double* Sqb = Sc + (long)qb * nn;
    // this wave's rows: r = w * IPW + p, i = iblk * IR + r

    for (int e = tid; e < 3 * IR * npt; e += NT) T1s[e] = 0.0;
    for (int e = tid; e < IR * npt; e += NT) {
        const int rr = e / npt, j = e - rr * npt;
        const int ii = iblk * IR + rr;
        Gbi[e] = (ii < n && j < n) ? Gb[(long)ii * n + j] : 0.0;
    }

    for (int j0 = 0; j0 < n; j0 += HT) {
        double xcol[IPW][TL];
#pragma unroll
        for (int p = 0; p < IPW; ++p)
#pragma unroll
            for (int c = 0; c < TL; ++c) xcol[p][c] = 0.0;
#pragma unroll 1
        for (int l0 = 0; l0 < n; l0 += HT) {
            double acc[IPW][TL][TL];
#pragma unroll
            for (int p = 0; p < IPW; ++p)
#pragma unroll
                for (int a = 0; a < TL; ++a)
#pragma unroll
                    for (int c = 0; c < TL; ++c) acc[p][a][c] = 0.0;
#pragma unroll 1
            for (int k0 = 0; k0 < n; k0 += VK) {
                __syncthreads();
                for (int e = tid; e < VK * HT; e += NT) {
                    const int kk = e / HT, jj = e - kk * HT;
                    const int k = k0 + kk, j = j0 + jj;
                    Bp[e] = (k < n && j < n) ? Gq[(long)k * n + j] : 0.0;
                }
                for (int e = tid; e < HT * VK; e += NT) {
                    const int ll = e / VK, kk = e - ll * VK;
                    const int l = l0 + ll, k = k0 + kk;
                    Ap[kk * HT + ll] = (l < n && k < n) ? Gb[(long)l * n + k] : 0.0;
                }
                for (int e = tid; e < IR * VK; e += NT) {
                    const int rr = e / VK, kk = e - rr * VK;
                    const int vi = iblk * IR + rr, k = k0 + kk;
                    Vp[e] = (vi < n && k < n) ? V[(long)vi * n + k] : 0.0;
                }
                __syncthreads();
                const int nk = min(VK, n - k0);
                const double* Vw = Vp + w * IPW * VK;
#pragma unroll 2
                for (int kk = 0; kk < nk; ++kk) {
                    double ar[TL], bv[TL];
#pragma unroll
                    for (int a = 0; a < TL; ++a) ar[a] = Ap[kk * HT + ty * TL + a];
#pragma unroll
                    for (int c = 0; c < TL; ++c) bv[c] = Bp[kk * HT + tx * TL + c];
#pragma unroll
                    for (int p = 0; p < IPW; ++p) {
                        const double vk = Vw[p * VK + kk];
#pragma unroll
                        for (int a = 0; a < TL; ++a) {
                            const double av = ar[a] * vk;
#pragma unroll
                            for (int c = 0; c < TL; ++c) acc[p][a][c] = fma(av, bv[c], acc[p][a][c]);
                        }
                    }
                }
            }
            // V rows l0.. and columns j0.. of this tile (zero outside n)
            __syncthreads();
            for (int e = tid; e < HT * HT; e += NT) {
                const int ll = e / HT, jj = e - ll * HT;
                const int l = l0 + ll, j = j0 + jj;
                Vt[ll * VLD + jj] = (l < n && j < n) ? V[(long)l * n + j] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < IPW; ++p) {
                const int rr = w * IPW + p, i = iblk * IR + rr;
                const bool iok = i < n;
                if (l0 == j0 && tx == ty) {
#pragma unroll
                    for (int a = 0; a < TL; ++a) T1s[rr * npt + l0 + ty * TL + a] = acc[p][a][a];
                }
                double gil[TL];
#pragma unroll
                for (int a = 0; a < TL; ++a) {
                    const int l = l0 + ty * TL + a;
                    gil[a] = (iok && l < n) ? Gq[(long)i * n + l] : 0.0;
                }
#pragma unroll
                for (int a = 0; a < TL; ++a) {
                    double s = 0.0;
#pragma unroll
                    for (int c = 0; c < TL; ++c) {
                        const double vm = Vt[(ty * TL + a) * VLD + tx * TL + c] * acc[p][a][c];
                        s += Gbi[rr * npt + j0 + tx * TL + c] * vm;
                        xcol[p][c] += gil[a] * vm;
                    }
                    // X'_il partial over this tile's columns: sum over the lane row (tx)
                    s += __shfl_xor(s, 1, 64);
                    s += __shfl_xor(s, 2, 64);
                    s += __shfl_xor(s, 4, 64);
                    if (tx == 0) XPs[rr * npt + l0 + ty * TL + a] += s;
                }
            }
        }
        // X_ij for this chunk's columns: sum over the lane column (ty)
#pragma unroll
        for (int p = 0; p < IPW; ++p)
#pragma unroll
            for (int c = 0; c < TL; ++c) {
                double s = xcol[p][c];
                s += __shfl_xor(s, 8, 64);
                s += __shfl_xor(s, 16, 64);
                s += __shfl_xor(s, 32, 64);
                if (ty == 0) Xs[(w * IPW + p) * npt + j0 + tx * TL + c] = s;
            }
    }

    // direct term D_ij = sum_l T1_il V_lj, then one store per output element
    for (int j0 = 0; j0 < n; j0 += 64) {
        double d[IPW];
#pragma unroll
        for (int p = 0; p < IPW; ++p) d[p] = 0.0;
        const int j = j0 + lane;
        for (int l0 = 0; l0 < n; l0 += 16) {
            __syncthreads();
            for (int e = tid; e < 16 * 64; e += NT) {
                const int ll = e >> 6, jj = e & 63;
                const int l = l0 + ll, jg = j0 + jj;
                Vt[ll * 65 + jj] = (l < n && jg < n) ? V[(long)l * n + jg] : 0.0;
            }
            __syncthreads();
#pragma unroll 4
            for (int ll = 0; ll < 16; ++ll) {
                const double vv = Vt[ll * 65 + lane];
#pragma unroll
                for (int p = 0; p < IPW; ++p) {
                    const double t = (l0 + ll < n) ? T1s[(w * IPW + p) * npt + l0 + ll] : 0.0;
                    d[p] = fma(t, vv, d[p]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < IPW; ++p) {
            const int rr = w * IPW + p, i = iblk * IR + rr;
            if (i < n && j < n) {
                const long ij = (long)i * n + j;
                Sq[ij] = sigma * Gq[ij] * d[p] - Xs[rr * npt + j];
                if (!middle) Sqb[ij] = sigma * Gb[ij] * d[p] - XPs[rr * npt + j];
            }
        }
    }
}

template <int IB, int TL, int IPW>
__global__ __launch_bounds__(IB * 64, (IB == 8 ? 4 : (IPW > 1 ? 2 : 3))) void k_sigma2b_valu(int n, int n_tau, int n_iblk,
                                                                             double sigma,
                                                                             const double* __restrict__ V,
                                                                             const double* __restrict__ G,
                                                                             double* __restrict__ Sc) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const long lb = xcd_remap(blockIdx.x, gridDim.x);
    s2b_tile_valu<IB, TL, IPW>(n, n_tau, (int)(lb / n_iblk), (int)(lb % n_iblk), sigma, V, G, Sc, smem_raw);
}

// One workgroup per (slice pair, block of IB rows i), XCD-aware block order.
template <int MODE, int IB, int JB, bool DB, int IPW>
__global__ __launch_bounds__(IB * 64, (waves_per_eu<MODE, IB, JB, DB, IPW>())) void k_sigma2b(
    int n, int n_tau, int n_iblk, typename Cfg<MODE>::T sigma, const typename Cfg<MODE>::T* __restrict__ V,
    const typename Cfg<MODE>::T* __restrict__ G, LowP lp, typename Cfg<MODE>::T* __restrict__ Sc) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const long lb = xcd_remap(blockIdx.x, gridDim.x);
    s2b_tile<MODE, IB, JB, DB, IPW>(n, n_tau, (int)(lb / n_iblk), (int)(lb % n_iblk), sigma, V, G, lp, Sc, smem_raw);
}

// One system of a batch for the persistent kernel. Its work items are
// item0 .. item0 + n_pairs * n_iblk - 1, ordered by slice pair, then row block.
template <class T>
struct S2BInst {
    const T* V;
    const T* G;
    T* Sc;
    LowP lp;
    long item0;
    T sigma;
    int n, n_iblk, n_pairs;
};

// Item ranges of the 8 per-XCD queues: queue x holds items [c[x], c[x+1]).
struct XcdCuts {
    long c[9];
};

// Persistent Sigma-2B over a batch of systems of different n_b (same n_tau).
// The grid is sized to the resident capacity of the chip; each workgroup takes
// items from the queue of its own XCD (consecutive items share a slice pair
// and so that XCD's L2), then steals from the other queues until all eight
// are empty. heads[0..7] count taken items per queue and must be zero at
// launch. Every workgroup leaves after eight failed probes.
template <int MODE, int IB, int JB, bool DB, int IPW>
__global__ __launch_bounds__(IB * 64, (waves_per_eu<MODE, IB, JB, DB, IPW>())) void k_sigma2b_batched(
    const S2BInst<typename Cfg<MODE>::T>* __restrict__ inst, int n_inst, int n_tau, XcdCuts cuts, int* heads) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ long s_item;
    const int x = blockIdx.x & 7;       // workgroups are dealt to the XCDs round-robin
    int probe = 0;
    while (probe < 8) {
        if (threadIdx.x == 0) {
            const int y = (x + probe) & 7;
            const long it = cuts.c[y] + atomicAdd(&heads[y], 1);
            s_item = it < cuts.c[y + 1] ? it : -1;
        }
        __syncthreads();
        const long it = s_item;
        __syncthreads();
        if (it < 0) {
            ++probe;
            continue;
        }
        int lo = 0, hi = n_inst - 1;    // last system with item0 <= it
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].item0 <= it) lo = mid;
            else hi = mid - 1;
        }
        const long local = it - inst[lo].item0;
        const int nib = inst[lo].n_iblk;
        s2b_tile<MODE, IB, JB, DB, IPW>(inst[lo].n, n_tau, (int)(local / nib), (int)(local % nib), inst[lo].sigma,
                                   inst[lo].V, inst[lo].G, inst[lo].lp, inst[lo].Sc, smem_raw);
    }
}

// The persistent loop of k_sigma2b_batched around the float64 vector-ALU tile.
template <int IB, int TL, int IPW>
__global__ __launch_bounds__(IB * 64, (IB == 8 ? 4 : (IPW > 1 ? 2 : 3))) void k_sigma2b_valu_batched(
    const S2BInst<double>* __restrict__ inst, int n_inst, int n_tau, XcdCuts cuts, int* heads) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ long s_item;
    const int x = blockIdx.x & 7;
    int probe = 0;
    while (probe < 8) {
        if (threadIdx.x == 0) {
            const int y = (x + probe) & 7;
            const long it = cuts.c[y] + atomicAdd(&heads[y], 1);
            s_item = it < cuts.c[y + 1] ? it : -1;
        }
        __syncthreads();
        const long it = s_item;
        __syncthreads();
        if (it < 0) {
            ++probe;
            continue;
        }
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].item0 <= it) lo = mid;
            else hi = mid - 1;
        }
        const long local = it - inst[lo].item0;
        const int nib = inst[lo].n_iblk;
        s2b_tile_valu<IB, TL, IPW>(inst[lo].n, n_tau, (int)(local / nib), (int)(local % nib), inst[lo].sigma, inst[lo].V,
                              inst[lo].G, inst[lo].Sc, smem_raw);
    }
}

__global__ void k_zero_int(int* p, int count) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = 0;
}

// ex[q] = e with 2^e max|G_q| in [1/2, 1) (0 for an all-zero slice)
__global__ __launch_bounds__(256) void k_slice_exponent(int n, const float* __restrict__ G, int* ex) {
    __shared__ float red[256];
    const long nn = (long)n * n;
    const float* g = G + (long)blockIdx.x * nn;
    float m = 0.f;
    for (long e = threadIdx.x; e < nn; e += 256) m = fmaxf(m, fabsf(g[e]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int e2 = 0;
        const float mx = red[0];
        if (mx > 0.f && isfinite(mx)) {
            frexpf(mx, &e2);          // mx = f 2^e2, f in [1/2, 1)
            e2 = -e2;
            if (e2 > 100) e2 = 100;
            if (e2 < -100) e2 = -100;
        }
        ex[blockIdx.x] = e2;
    }
}

// gh[q][j][k] = bf16(G_q[j][k] 2^ex[q]) for k < n, 0 for n <= k < ldb; one
// 16-byte piece (8 values of k) per thread, grid (pieces / 256, n_tau)
__global__ __launch_bounds__(256) void k_slice_bf16(int n, int ldb, const float* __restrict__ G,
                                                    const int* __restrict__ ex, __bf16* __restrict__ gh) {
    const int q = blockIdx.y;
    const int per_row = ldb / 8;
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v >= (long)n * per_row) return;
    const int j = (int)(v / per_row), k0 = 8 * (int)(v % per_row);
    const float sc = ldexpf(1.0f, ex[q]);
    const float* g = G + (long)q * n * n + (long)j * n;
    bf16x8 out;
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = (__bf16)(k0 + e < n ? g[k0 + e] * sc : 0.0f);
    *reinterpret_cast<bf16x8*>(gh + ((long)q * n + j) * ldb + k0) = out;
}

int bf16_ldb(int n) { return (n + 7) & ~7; }

// The bf16 copy of every slice (after k_slice_exponent has filled ex).
int slices_to_bf16(int n, int n_tau, const float* G, const int* ex, __bf16* gh, hipStream_t st) {
    const long pieces = (long)n * (bf16_ldb(n) / 8);
    const long gx = (pieces + 255) / 256;
    if (gx > 0x7fffffffL || n_tau > 65535) {
        set_error("Sigma-2B bf16 staging: %d slices of n_b = %d exceed the launch limits", n_tau, n);
        return NEGF_EINVAL;
    }
    hipLaunchKernelGGL(k_slice_bf16, dim3((unsigned)gx, (unsigned)n_tau), dim3(256), 0, st, n, bf16_ldb(n), G, ex,
                       gh);
    LAUNCH_CHECK();
    return NEGF_OK;
}

// Tile configurations the tuner chooses from: waves per workgroup (one value
// of i each unless noted) and 16-wide column blocks per chunk.
// 0: 8 x 208 cols, 1: 8 x 112, 2: 4 x 208, 3: 4 x 112 (single-buffered staging);
// 4: 8 x 112, 5: 8 x 208 (double-buffered staging);
// 6: 4 waves x 2 values of i x 112 cols, 7: 4 x 2 x 64 cols (float32 and bf16 only);
// 8: 8 waves x 40 x 40 vector-ALU tiles, 9: 4 waves x 2 values of i x 40 x 40,
// 10: 4 x 2 x 32 x 32 (float64 only); 11, 12: 8 or 4 waves x 208 columns with
// direct-to-LDS double-buffered staging from padded copies (float64 only, not
// in the persistent kernel).
constexpr int kNumCfg = 13;

// float64 tile with direct-to-LDS staging: zero-padded copies of G and V in
// context scratch (one pass each per call), then one workgroup per (slice pair,
// block of IB rows i).
template <int IB, int JB, int BK>
int launch_dma_cfg(negf_ctx* ctx, int n, int n_tau, int sigma, const double* V, const double* G, double* Sc,
                   hipStream_t st) {
    const int np = (n + 15) & ~15;
    const size_t smem = dma::Layout<IB, JB, BK>::bytes(np);
    if (smem > 160 * 1024) {
        set_error("n_b = %d too large for this Sigma-2B tile configuration's LDS budget", n);
        return NEGF_EINVAL;
    }
    const int n_pairs = (n_tau + 1) / 2;
    const int n_iblk = (n + IB - 1) / IB;
    // an odd n_tau has a middle slice: split over up to 8 parts of its l-tiles
    const int n_parts = (n_tau & 1) && n_pairs >= 2 ? std::min(8, (n + 15) / 16) : 0;
    const long n_full = (long)(n_parts ? n_pairs - 1 : n_pairs) * n_iblk;
    const long blocks = n_full + (long)n_parts * n_iblk;
    if (blocks > 0x7fffffffL) {
        set_error("too many workgroups");
        return NEGF_EINVAL;
    }
    const long ni = (long)n_iblk * IB * np;
    double* part = nullptr;
    if (n_parts) NEGF_TRY(scratch_t(ctx, "s2b_parts", (size_t)2 * ni * n_parts, &part));
    double *Gp = nullptr, *Vp = nullptr;
    NEGF_TRY(scratch_t(ctx, "s2b_gpad", (size_t)n_tau * np * np, &Gp));
    NEGF_TRY(scratch_t(ctx, "s2b_vpad", (size_t)np * np, &Vp));
    auto pad = [&](const double* src, double* dst, long count) -> int {
        if (count <= 0) return NEGF_OK;
        const unsigned bx = (unsigned)std::min<long>(((long)np * np / 2 + 255) / 256, 1024);
        const unsigned by = (unsigned)std::min<long>(count, 65535);
        hipLaunchKernelGGL(k_pad_copy, dim3(bx, by), dim3(256), 0, st, n, np, count, src, dst);
        LAUNCH_CHECK();
        return NEGF_OK;
    };
    NEGF_TRY(pad(G, Gp, n_tau));
    NEGF_TRY(pad(V, Vp, 1));
    static bool attr_set = false;
    if (!attr_set) {
        HIP_TRY(hipFuncSetAttribute((const void*)k_sigma2b_dma<IB, JB, BK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_sigma2b_dma<IB, JB, BK>), dim3((unsigned)blocks), dim3(IB * 64), smem, st, n, np, n_tau, n_iblk,
                       (double)sigma, Vp, Gp, G, Sc, n_full, n_parts, part);
    LAUNCH_CHECK();
    if (n_parts) {
        const long q = (n_tau - 1) / 2, nn = (long)n * n;
        hipLaunchKernelGGL(k_s2b_parts_sum, dim3((unsigned)std::min<long>((nn + 255) / 256, 4096)), dim3(256), 0, st, n,
                           np, ni, n_parts, (double)sigma, G + q * nn, part, Sc + q * nn);
        LAUNCH_CHECK();
    }
    return NEGF_OK;
}

template <int IB, int TL, int IPW>
int launch_valu_cfg(int n, int n_tau, int sigma, const double* V, const double* G, double* Sc, hipStream_t st) {
    const int n_pairs = (n_tau + 1) / 2;
    const int n_iblk = (n + IB * IPW - 1) / (IB * IPW);
    const size_t smem = lds_bytes_valu<IB, TL, IPW>(n);
    if (smem > 160 * 1024) {
        set_error("n_b = %d too large for this Sigma-2B tile configuration's LDS budget", n);
        return NEGF_EINVAL;
    }
    const long blocks = (long)n_pairs * n_iblk;
    if (blocks > 0x7fffffffL) {
        set_error("too many workgroups");
        return NEGF_EINVAL;
    }
    static bool attr_set = false;
    if (!attr_set) {
        HIP_TRY(hipFuncSetAttribute((const void*)k_sigma2b_valu<IB, TL, IPW>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_sigma2b_valu<IB, TL, IPW>), dim3((unsigned)blocks), dim3(IB * 64), smem, st, n, n_tau, n_iblk,
                       (double)sigma, V, G, Sc);
    LAUNCH_CHECK();
    return NEGF_OK;
}

template <int MODE, int IB, int JB, bool DB, int IPW>
int launch_cfg(int n, int n_tau, int sigma, const typename Cfg<MODE>::T* V, const typename Cfg<MODE>::T* G,
               LowP lp, typename Cfg<MODE>::T* Sc, hipStream_t st) {
    typedef typename Cfg<MODE>::T T;
    const int n_pairs = (n_tau + 1) / 2;
    const int n_iblk = (n + IB * IPW - 1) / (IB * IPW);
    const int np = (n + 15) & ~15;
    const size_t smem = lds_bytes<MODE, IB, JB, DB, IPW>(np);
    if (smem > 160 * 1024) {
        set_error("n_b = %d too large for the Sigma-2B kernel's LDS budget", n);
        return NEGF_EINVAL;
    }
    const long blocks = (long)n_pairs * n_iblk;
    if (blocks > 0x7fffffffL) {
        set_error("too many workgroups");
        return NEGF_EINVAL;
    }
    static bool attr_set = false;
    if (!attr_set) {
        HIP_TRY(hipFuncSetAttribute((const void*)k_sigma2b<MODE, IB, JB, DB, IPW>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_sigma2b<MODE, IB, JB, DB, IPW>), dim3((unsigned)blocks), dim3(IB * 64), smem, st, n, n_tau, n_iblk,
                       T(sigma), V, G, lp, Sc);
    LAUNCH_CHECK();
    return NEGF_OK;
}

// ex_fixed (nullable): caller-provided storage for the per-slice exponents of
// the low-precision modes (at least n_tau ints); otherwise context scratch.
template <int MODE>
int launch(negf_ctx* ctx, int n, int n_tau, int sigma, const typename Cfg<MODE>::T* V,
           const typename Cfg<MODE>::T* G, typename Cfg<MODE>::T* Sc, int cfg, hipStream_t st,
           int* ex_fixed = nullptr) {
    int* ex = ex_fixed;
    LowP lp{nullptr, nullptr, 0};
    if (MODE != MODE_F64) {
        if (!ex) NEGF_TRY(scratch_t(ctx, "s2b_ex", n_tau, &ex));
        hipLaunchKernelGGL(k_slice_exponent, dim3(n_tau), dim3(256), 0, st, n, (const float*)G, ex);
        LAUNCH_CHECK();
        lp.ex = ex;
    }
    if (MODE == MODE_BF16) {
        __bf16* gh = nullptr;
        NEGF_TRY(scratch_t(ctx, "s2b_gh", (size_t)n_tau * n * bf16_ldb(n), &gh));
        NEGF_TRY(slices_to_bf16(n, n_tau, (const float*)G, ex, gh, st));
        lp.gh = gh;
        lp.ldb = bf16_ldb(n);
    }
    switch (cfg) {
        case 0: return launch_cfg<MODE, 8, 13, false, 1>(n, n_tau, sigma, V, G, lp, Sc, st);
        case 1: return launch_cfg<MODE, 8, 7, false, 1>(n, n_tau, sigma, V, G, lp, Sc, st);
        case 2: return launch_cfg<MODE, 4, 13, false, 1>(n, n_tau, sigma, V, G, lp, Sc, st);
        case 3: return launch_cfg<MODE, 4, 7, false, 1>(n, n_tau, sigma, V, G, lp, Sc, st);
        case 4: return launch_cfg<MODE, 8, 7, true, 1>(n, n_tau, sigma, V, G, lp, Sc, st);
        case 5: return launch_cfg<MODE, 8, 13, true, 1>(n, n_tau, sigma, V, G, lp, Sc, st);
        default:
            if constexpr (MODE == MODE_F64) {
                const double* Vd = (const double*)V;
                const double* Gd = (const double*)G;
                double* Sd = (double*)Sc;
                if (cfg == 8) return launch_valu_cfg<8, 5, 1>(n, n_tau, sigma, Vd, Gd, Sd, st);
                if (cfg == 9) return launch_valu_cfg<4, 5, 2>(n, n_tau, sigma, Vd, Gd, Sd, st);
                if (cfg == 10) return launch_valu_cfg<4, 4, 2>(n, n_tau, sigma, Vd, Gd, Sd, st);
                if (cfg == 11) return launch_dma_cfg<8, 13, 16>(ctx, n, n_tau, sigma, Vd, Gd, Sd, st);
                if (cfg == 12) return launch_dma_cfg<4, 13, 4>(ctx, n, n_tau, sigma, Vd, Gd, Sd, st);
                set_error("tile configuration %d is for float32 and bf16 only", cfg);
                return NEGF_EINVAL;
            } else {
                if (cfg == 6) return launch_cfg<MODE, 4, 7, false, 2>(n, n_tau, sigma, V, G, lp, Sc, st);
                if (cfg == 7) return launch_cfg<MODE, 4, 4, false, 2>(n, n_tau, sigma, V, G, lp, Sc, st);
                set_error("tile configuration %d is for float64 only", cfg);
                return NEGF_EINVAL;
            }
    }
}

// Default before tuning: the narrower column chunk keeps the accumulators small
// enough for two workgroups per CU.
int default_cfg(int mode, int n) {
    (void)mode;
    (void)n;
    return 1;
}

std::string tune_key(int mode, int n) { return "s2b_cfg_" + std::to_string(mode) + "_" + std::to_string(n); }

}  // namespace

int sigma2b_set_cfg(negf_ctx* ctx, int dtype, int n, int cfg) {
    if (cfg < 0 || cfg >= kNumCfg) {
        set_error("tile configuration %d out of range [0, %d)", cfg, kNumCfg);
        return NEGF_EINVAL;
    }
    const int mode = dtype == NEGF_F64 ? MODE_F64 : (dtype == NEGF_BF16 ? MODE_BF16 : MODE_F32);
    ctx->filled[tune_key(mode, n)] = cfg;
    return NEGF_OK;
}

namespace {

}  // namespace

template <class T>
int sigma2b_cfg(negf_ctx* ctx, int n, int n_tau, int sigma, const T* V, const T* G, T* Sc, bool bf16, int cfg,
                hipStream_t st, int* ex_fixed = nullptr);

template <class T>
int sigma2b_run(negf_ctx* ctx, int n, int n_tau, int sigma, const T* V, const T* G, T* Sc, bool bf16,
                hipStream_t st) {
    const int mode = sizeof(T) == 8 ? MODE_F64 : (bf16 ? MODE_BF16 : MODE_F32);
    auto it = ctx->filled.find(tune_key(mode, n));
    const int cfg = it != ctx->filled.end() ? it->second : default_cfg(mode, n);
    return sigma2b_cfg<T>(ctx, n, n_tau, sigma, V, G, Sc, bf16, cfg, st);
}

template <class T>
int sigma2b_cfg(negf_ctx* ctx, int n, int n_tau, int sigma, const T* V, const T* G, T* Sc, bool bf16, int cfg,
                hipStream_t st, int* ex_fixed) {
    if (sizeof(T) == 8) return launch<MODE_F64>(ctx, n, n_tau, sigma, (const double*)V, (const double*)G, (double*)Sc, cfg, st);
    if (bf16) return launch<MODE_BF16>(ctx, n, n_tau, sigma, (const float*)V, (const float*)G, (float*)Sc, cfg, st);
    return launch<MODE_F32>(ctx, n, n_tau, sigma, (const float*)V, (const float*)G, (float*)Sc, cfg, st, ex_fixed);
}

// Float64 Sigma-2B of one system: the configuration tuned for (float64, n_b) in
// this context, else the direct-to-LDS tile with 8 values of i (configuration
// 11) where its LDS fits n_b, else the default. Stream-ordered; after its first
// call for a size (scratch, kernel attribute) it may be captured in a graph.
int sigma2b_run_f64_single(negf_ctx* ctx, int n, int n_tau, int sigma, const double* V, const double* G, double* Sc,
                           hipStream_t st) {
    auto it = ctx->filled.find(tune_key(MODE_F64, n));
    int cfg = default_cfg(MODE_F64, n);
    if (it != ctx->filled.end()) cfg = it->second;
    else if (dma::Layout<8, 13, 16>::bytes((n + 15) & ~15) <= 160 * 1024) cfg = 11;
    return sigma2b_cfg<double>(ctx, n, n_tau, sigma, V, G, Sc, false, cfg, st);
}

// ---------------------------------------------------------------- allocation-free entry
// The per-slice exponents of the float32 mode live in a fixed device array for
// callers that cannot allocate (one copy per GPU, kept until the process ends).
// Host code never passes the array's name to a kernel: each device's address
// comes from hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) int s2b_noalloc_ex[NEGF_SIGMA2B_NOALLOC_MAX_TAU];

namespace {
std::mutex g_noalloc_mu;
std::vector<int*> g_noalloc_ptr;      // per device id
}  // namespace

int s2b_noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if ((int)g_noalloc_ptr.size() <= device) g_noalloc_ptr.resize(device + 1, nullptr);
    if (g_noalloc_ptr[device]) return NEGF_OK;
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(s2b_noalloc_ex)));
    g_noalloc_ptr[device] = static_cast<int*>(p);
    return NEGF_OK;
}

template <class T>
int sigma2b_run_noalloc(negf_ctx* ctx, int n, int n_tau, int sigma, const T* V, const T* G, T* Sc, hipStream_t st) {
    int* ex = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (ctx->device < (int)g_noalloc_ptr.size()) ex = g_noalloc_ptr[ctx->device];
    }
    if (!ex) {
        set_error("allocation-free Sigma-2B: device %d was not set up by negf_ctx_create", ctx->device);
        return NEGF_EHIP;
    }
    const int mode = sizeof(T) == 8 ? MODE_F64 : MODE_F32;
    auto it = ctx->filled.find(tune_key(mode, n));
    int cfg = it != ctx->filled.end() ? it->second : default_cfg(mode, n);
    // the configurations that stage through padded copies need scratch: the
    // 208-column matrix-core tile stands in for them
    if (cfg >= 11) cfg = 0;
    return sigma2b_cfg<T>(ctx, n, n_tau, sigma, V, G, Sc, false, cfg, st, ex);
}
template int sigma2b_run_noalloc<double>(negf_ctx*, int, int, int, const double*, const double*, double*, hipStream_t);
template int sigma2b_run_noalloc<float>(negf_ctx*, int, int, int, const float*, const float*, float*, hipStream_t);

// Time every tile configuration on the caller's input (after one untimed
// launch each) and remember the fastest for (mode, n_b) in the context.
template <class T>
int sigma2b_tune(negf_ctx* ctx, int n, int n_tau, int sigma, const T* V, const T* G, T* Sc, bool bf16, int* best,
                 double* ms, hipStream_t st) {
    const int mode = sizeof(T) == 8 ? MODE_F64 : (bf16 ? MODE_BF16 : MODE_F32);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int arg = -1;
    float tbest = 0.f;
    for (int c = 0; c < kNumCfg; ++c) {
        int rc = sigma2b_cfg<T>(ctx, n, n_tau, sigma, V, G, Sc, bf16, c, st);
        if (rc == NEGF_EINVAL) {          // configuration does not fit this n_b
            if (ms) ms[c] = -1.0;
            continue;
        }
        NEGF_TRY(rc);
        HIP_TRY(hipEventRecord(e0, st));
        NEGF_TRY(sigma2b_cfg<T>(ctx, n, n_tau, sigma, V, G, Sc, bf16, c, st));
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        if (ms) ms[c] = t;
        if (arg < 0 || t < tbest) {
            arg = c;
            tbest = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (arg < 0) {
        set_error("no Sigma-2B tile configuration fits n_b = %d", n);
        return NEGF_EINVAL;
    }
    ctx->filled[tune_key(mode, n)] = arg;
    if (best) *best = arg;
    return NEGF_OK;
}

// ============================================================== batched (persistent) form
namespace {

template <int MODE, int IB, int JB, bool DB, int IPW>
int launch_batched_cfg(const S2BBatch& pl, hipStream_t st) {
    typedef typename Cfg<MODE>::T T;
    const int np = (pl.max_n + 15) & ~15;
    const size_t smem = lds_bytes<MODE, IB, JB, DB, IPW>(np);
    if (smem + 64 > 160 * 1024) {
        set_error("n_b = %d too large for this Sigma-2B tile configuration's LDS budget", pl.max_n);
        return NEGF_EINVAL;
    }
    auto kern = k_sigma2b_batched<MODE, IB, JB, DB, IPW>;
    static bool attr_set = false;
    if (!attr_set) {
        HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 64));
        attr_set = true;
    }
    int occ = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, IB * 64, smem));
    if (occ < 1) {
        set_error("Sigma-2B tile configuration does not fit a compute unit at n_b = %d", pl.max_n);
        return NEGF_EINVAL;
    }
    long grid = (long)occ * pl.n_cu;
    if (grid > pl.n_items) grid = pl.n_items;
    if (grid < 1) return NEGF_OK;
    XcdCuts cuts;
    for (int x = 0; x < 9; ++x) cuts.c[x] = pl.cuts[x];
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, pl.heads, 8);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(IB * 64), smem, st,
                       (const S2BInst<T>*)pl.d_inst, pl.n_inst, pl.n_tau, cuts, pl.heads);
    LAUNCH_CHECK();
    return NEGF_OK;
}

template <int IB, int TL, int IPW>
int launch_batched_valu_cfg(const S2BBatch& pl, hipStream_t st) {
    const size_t smem = lds_bytes_valu<IB, TL, IPW>(pl.max_n);
    if (smem + 64 > 160 * 1024) {
        set_error("n_b = %d too large for this Sigma-2B tile configuration's LDS budget", pl.max_n);
        return NEGF_EINVAL;
    }
    auto kern = k_sigma2b_valu_batched<IB, TL, IPW>;
    static bool attr_set = false;
    if (!attr_set) {
        HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 64));
        attr_set = true;
    }
    int occ = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, IB * 64, smem));
    if (occ < 1) {
        set_error("Sigma-2B tile configuration does not fit a compute unit at n_b = %d", pl.max_n);
        return NEGF_EINVAL;
    }
    long grid = (long)occ * pl.n_cu;
    if (grid > pl.n_items) grid = pl.n_items;
    if (grid < 1) return NEGF_OK;
    XcdCuts cuts;
    for (int x = 0; x < 9; ++x) cuts.c[x] = pl.cuts[x];
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, pl.heads, 8);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(IB * 64), smem, st, (const S2BInst<double>*)pl.d_inst,
                       pl.n_inst, pl.n_tau, cuts, pl.heads);
    LAUNCH_CHECK();
    return NEGF_OK;
}

template <int MODE>
int launch_batched(const S2BBatch& pl, int cfg, hipStream_t st) {
    switch (cfg) {
        case 0: return launch_batched_cfg<MODE, 8, 13, false, 1>(pl, st);
        case 1: return launch_batched_cfg<MODE, 8, 7, false, 1>(pl, st);
        case 2: return launch_batched_cfg<MODE, 4, 13, false, 1>(pl, st);
        case 3: return launch_batched_cfg<MODE, 4, 7, false, 1>(pl, st);
        case 4: return launch_batched_cfg<MODE, 8, 7, true, 1>(pl, st);
        case 5: return launch_batched_cfg<MODE, 8, 13, true, 1>(pl, st);
        default:
            if constexpr (MODE == MODE_F64) {
                if (cfg == 8) return launch_batched_valu_cfg<8, 5, 1>(pl, st);
                if (cfg == 9) return launch_batched_valu_cfg<4, 5, 2>(pl, st);
                if (cfg == 10) return launch_batched_valu_cfg<4, 4, 2>(pl, st);
                if (cfg == 11 || cfg == 12) {
                    set_error("tile configuration %d (staged padded copies) is not available in the persistent kernel",
                              cfg);
                    return NEGF_EINVAL;
                }
                set_error("tile configuration %d is for float32 and bf16 only", cfg);
                return NEGF_EINVAL;
            } else {
                if (cfg == 6) return launch_batched_cfg<MODE, 4, 7, false, 2>(pl, st);
                if (cfg == 7) return launch_batched_cfg<MODE, 4, 4, false, 2>(pl, st);
                set_error("tile configuration %d is for float64 only", cfg);
                return NEGF_EINVAL;
            }
    }
}

// rows i per workgroup of a configuration
int cfg_rows(int cfg) { return (cfg == 2 || cfg == 3) ? 4 : 8; }

std::string batch_key(int mode, const std::vector<int>& n) {
    std::string k = "s2bB_" + std::to_string(mode);
    for (int v : n) k += "_" + std::to_string(v);
    return k;
}

template <class T>
int prepare_typed(negf_ctx* ctx, const std::string& tag, int batch, const int* n, int n_tau, const int* sigma,
                  const void* const* V, const void* const* G, void* const* Sc, int pair_lim, S2BBatch* pl,
                  hipStream_t st) {
    // systems in order of decreasing n_b: the largest items are taken first
    std::vector<int> order(batch);
    for (int b = 0; b < batch; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
    const int rows = cfg_rows(pl->cfg);
    const int n_pairs_all = (n_tau + 1) / 2;
    const int n_pairs = pair_lim > 0 && pair_lim < n_pairs_all ? pair_lim : n_pairs_all;
    std::vector<S2BInst<T>> hi(batch);
    std::vector<double> cost(batch);
    int* ex = nullptr;
    if (pl->mode != MODE_F64) NEGF_TRY(scratch_t(ctx, ("s2bB_ex_" + tag).c_str(), (size_t)batch * n_tau, &ex));
    __bf16* gh = nullptr;
    if (pl->mode == MODE_BF16) {
        size_t tot = 0;
        for (int b = 0; b < batch; ++b) tot += (size_t)n_tau * n[b] * bf16_ldb(n[b]);
        NEGF_TRY(scratch_t(ctx, ("s2bB_gh_" + tag).c_str(), tot, &gh));
    }
    size_t gh_off = 0;
    long items = 0;
    double total = 0.0;
    pl->n_sorted.assign(batch, 0);
    pl->G_sorted.assign(batch, nullptr);
    pl->ex_sorted.assign(batch, nullptr);
    pl->gh_sorted.assign(batch, nullptr);
    pl->max_n = 0;
    for (int r = 0; r < batch; ++r) {
        const int b = order[r];
        S2BInst<T>& I = hi[r];
        I.V = (const T*)V[b];
        I.G = (const T*)G[b];
        I.Sc = (T*)Sc[b];
        I.lp.ex = ex ? ex + (long)r * n_tau : nullptr;
        I.lp.gh = gh ? gh + gh_off : nullptr;
        I.lp.ldb = gh ? bf16_ldb(n[b]) : 0;
        pl->gh_sorted[r] = gh ? gh + gh_off : nullptr;
        if (gh) gh_off += (size_t)n_tau * n[b] * bf16_ldb(n[b]);
        I.item0 = items;
        I.sigma = (T)sigma[b];
        I.n = n[b];
        I.n_iblk = (n[b] + rows - 1) / rows;
        I.n_pairs = n_pairs;
        items += (long)n_pairs * I.n_iblk;
        cost[r] = (double)n[b] * n[b] * n[b];
        total += cost[r] * n_pairs * I.n_iblk;
        pl->n_sorted[r] = n[b];
        pl->G_sorted[r] = G[b];
        pl->ex_sorted[r] = ex ? ex + (long)r * n_tau : nullptr;
        if (n[b] > pl->max_n) pl->max_n = n[b];
    }
    // equal-cost contiguous item ranges, one per XCD
    pl->cuts.assign(9, items);
    pl->cuts[0] = 0;
    double acc = 0.0;
    int x = 1;
    for (int r = 0; r < batch && x < 8; ++r) {
        const long cnt = (long)n_pairs * hi[r].n_iblk;
        const double seg = cost[r] * cnt;
        while (x < 8 && acc + seg >= total * x / 8.0) {
            long off = (long)std::ceil((total * x / 8.0 - acc) / cost[r]);
            if (off > cnt) off = cnt;
            if (off < 0) off = 0;
            pl->cuts[x] = hi[r].item0 + off;
            ++x;
        }
        acc += seg;
    }
    for (int y = 1; y < 9; ++y)
        if (pl->cuts[y] < pl->cuts[y - 1]) pl->cuts[y] = pl->cuts[y - 1];
    pl->n_inst = batch;
    pl->n_tau = n_tau;
    pl->n_items = items;
    NEGF_TRY(upload(ctx, ("s2bB_inst_" + tag).c_str(), hi.data(), sizeof(S2BInst<T>) * batch, st, &pl->d_inst));
    NEGF_TRY(scratch_t(ctx, ("s2bB_heads_" + tag).c_str(), 8, &pl->heads));
    return NEGF_OK;
}

}  // namespace

int s2b_batch_prepare(negf_ctx* ctx, const char* tag, int dtype, int batch, const int* n, int n_tau,
                      const int* sigma, const void* const* V, const void* const* G, void* const* Sc, int pair_lim,
                      S2BBatch* pl, hipStream_t st) {
    pl->mode = dtype == NEGF_F64 ? MODE_F64 : (dtype == NEGF_BF16 ? MODE_BF16 : MODE_F32);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&pl->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    std::vector<int> ns(n, n + batch);
    std::sort(ns.begin(), ns.end());
    pl->key = batch_key(pl->mode, ns);
    if (pl->cfg < 0) {
        auto it = ctx->filled.find(pl->key);
        pl->cfg = it != ctx->filled.end() ? it->second : default_cfg(pl->mode, 0);
    }
    const std::string t(tag);
    if (pl->mode == MODE_F64)
        return prepare_typed<double>(ctx, t, batch, n, n_tau, sigma, V, G, Sc, pair_lim, pl, st);
    return prepare_typed<float>(ctx, t, batch, n, n_tau, sigma, V, G, Sc, pair_lim, pl, st);
}

// Stream-ordered and free of host synchronisation: may be captured in a graph.
int s2b_batch_launch(const S2BBatch& pl, hipStream_t st) {
    if (pl.mode != MODE_F64) {
        for (int r = 0; r < pl.n_inst; ++r) {
            hipLaunchKernelGGL(k_slice_exponent, dim3(pl.n_tau), dim3(256), 0, st, pl.n_sorted[r],
                               (const float*)pl.G_sorted[r], pl.ex_sorted[r]);
            LAUNCH_CHECK();
            if (pl.mode == MODE_BF16)
                NEGF_TRY(slices_to_bf16(pl.n_sorted[r], pl.n_tau, (const float*)pl.G_sorted[r], pl.ex_sorted[r],
                                        (__bf16*)pl.gh_sorted[r], st));
        }
    }
    if (pl.mode == MODE_F64) return launch_batched<MODE_F64>(pl, pl.cfg, st);
    if (pl.mode == MODE_BF16) return launch_batched<MODE_BF16>(pl, pl.cfg, st);
    return launch_batched<MODE_F32>(pl, pl.cfg, st);
}

// Tile autotuner for a batch: every configuration is timed on the first
// pair_lim slice pairs of every system (the same mix of n_b as the full run),
// and the fastest is stored for this multiset of n_b.
int s2b_batch_tune(negf_ctx* ctx, int dtype, int batch, const int* n, int n_tau, const int* sigma,
                   const void* const* V, const void* const* G, void* const* Sc, int pair_lim, int* best, double* ms,
                   hipStream_t st) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int arg = -1;
    float tbest = 0.f;
    std::string key;
    for (int c = 0; c < kNumCfg; ++c) {
        S2BBatch pl;
        pl.cfg = c;
        NEGF_TRY(s2b_batch_prepare(ctx, "tune", dtype, batch, n, n_tau, sigma, V, G, Sc, pair_lim, &pl, st));
        key = pl.key;
        int rc = s2b_batch_launch(pl, st);
        if (rc == NEGF_EINVAL) {
            if (ms) ms[c] = -1.0;
            continue;
        }
        NEGF_TRY(rc);
        HIP_TRY(hipEventRecord(e0, st));
        NEGF_TRY(s2b_batch_launch(pl, st));
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        if (ms) ms[c] = t;
        if (arg < 0 || t < tbest) {
            arg = c;
            tbest = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (arg < 0) {
        set_error("no Sigma-2B tile configuration fits this batch");
        return NEGF_EINVAL;
    }
    ctx->filled[key] = arg;
    if (best) *best = arg;
    return NEGF_OK;
}

template int sigma2b_tune<double>(negf_ctx*, int, int, int, const double*, const double*, double*, bool, int*, double*, hipStream_t);
template int sigma2b_tune<float>(negf_ctx*, int, int, int, const float*, const float*, float*, bool, int*, double*, hipStream_t);

template int sigma2b_run<double>(negf_ctx*, int, int, int, const double*, const double*, double*, bool, hipStream_t);
template int sigma2b_run<float>(negf_ctx*, int, int, int, const float*, const float*, float*, bool, hipStream_t);

}  // namespace negf
