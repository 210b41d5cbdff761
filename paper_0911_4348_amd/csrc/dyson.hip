// One step of the Matsubara Dyson equation and the Galitskii-Migdal energy
// (paper Sec. 2.3, Eq. deq and the text after it).
//
//   rho = -G(beta^-),  St = Sigma^HF[rho] - Sigma0
//   I1_p = St G_p + Q_p[Sigma_c, G],  I2_p = Q_p[G0, I1],
//   G_out = (1 - alpha) G_in + alpha (G0 + I2),  optionally (G + G^T)/2.
//
// Q is the split trapezoid rule: the integral over [0, beta] is split at tau_p
// and each part uses the trapezoid rule on the grid points it covers, with the
// antiperiodic continuation A(s - beta) = -A(s) and one-sided values at the
// split point.
//
// Q[Sigma_c, G]: on a uniform grid with M = 2^L intervals, for 0 < p < M the
// sum is an antiperiodic circular convolution of length M (jump averages at
// q = 0); it is computed through the DFT at the odd Matsubara frequencies:
// real columns are packed in pairs, twisted by e^(-i pi q / M) and transformed
// in LDS, the static term St enters as a frequency-independent addition, and
// p = 0, M are corrected with one n_b x n_b product. Any grid (and the power
// mesh, with 4-point Lagrange interpolation of Sigma_c inside its uniform
// block) can use the direct double sum on the matrix cores instead.
//
// Q[G0, I1]: in the HF eigenbasis G0 is diagonal, G0 = -C diag(g(tau)) C^T,
// g_k(s) = (1 - f_k) e^(-s xi_k), so each (k, column) pair needs two
// first-order recurrences over tau, arranged so that every exponential factor
// is <= 1 (forward decay or a prefix sum with e^(xi tau) for xi < 0, and the
// mirror images backwards). G0 itself is added in the same pass.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "common.h"
#include "mfma.h"

namespace negf {
namespace {

inline unsigned grid_for(long total) {
    long b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Compensated (Neumaier) float64 sum: the value is s + c, where c gathers the
// rounding error of every addition into s (exact for each addition, since the
// error of a rounded sum of two doubles is itself a double). Merging two such
// sums adds the partner's s the same way and its c plainly; the merge is
// symmetric, so every lane of a butterfly ends with the same pair.
struct CSum {
    double s, c;
    __device__ void add(double x) {
#pragma clang fp contract(off)
        const double t = s + x;
        c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    __device__ void merge(double os, double oc) {
        add(os);
        c += oc;
    }
    __device__ double value() const { return s + c; }
};

// Block-wide compensated sum, in a fixed order (waves by butterfly, then the
// waves' partial sums in wave order by thread 0), as the unrounded pair (sum,
// compensation), valid in thread 0. red holds 2 (NT/64) + 2 doubles.
template <int NT>
__device__ CSum block_csum_pair(CSum v, double* red) {
    for (int off = 32; off > 0; off >>= 1) {
        const double os = __shfl_xor(v.s, off, 64), oc = __shfl_xor(v.c, off, 64);
        v.merge(os, oc);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) {
        red[2 * w] = v.s;
        red[2 * w + 1] = v.c;
    }
    __syncthreads();
    CSum t{red[0], red[1]};
    if (threadIdx.x == 0)
        for (int k = 1; k < NT / 64; ++k) t.merge(red[2 * k], red[2 * k + 1]);
    __syncthreads();
    return t;
}

// The same rounded to one double, returned to every thread.
template <int NT>
__device__ double block_csum(CSum v, double* red) {
    for (int off = 32; off > 0; off >>= 1) {
        const double os = __shfl_xor(v.s, off, 64), oc = __shfl_xor(v.c, off, 64);
        v.merge(os, oc);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) {
        red[2 * w] = v.s;
        red[2 * w + 1] = v.c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        CSum t{red[0], red[1]};
        for (int k = 1; k < NT / 64; ++k) t.merge(red[2 * k], red[2 * k + 1]);
        red[2 * (NT / 64)] = t.value();
    }
    __syncthreads();
    return red[2 * (NT / 64)];
}


// ------------------------------------------------------------ St = Sigma^HF[-G_M] - Sigma0
// (with Lm, Rm given, also the end-point matrices of the Fourier route)
template <class T>
__global__ __launch_bounds__(256) void k_sigma_tilde(int n, int sigma, const double* __restrict__ V,
                                                     const T* __restrict__ GM, const double* __restrict__ Sigma0,
                                                     T* __restrict__ St, T dtau, const T* __restrict__ Sc0,
                                                     const T* __restrict__ ScM, const T* __restrict__ G0,
                                                     T* __restrict__ Lm, T* __restrict__ Rm) {
    __shared__ double red[2 * 4 + 2];
    const int i = blockIdx.x;                           // one workgroup per row
    if (i >= n) return;
    const long r = (long)i * n;
    // Hartree term of row i: sum over k of V_ik rho_kk, rho = -G_M
    CSum hs{0.0, 0.0};
    for (int k = threadIdx.x; k < n; k += 256) hs.add(-V[r + k] * (double)GM[(long)k * n + k]);
    const double h = block_csum<256>(hs, red);
    for (int j = threadIdx.x; j < n; j += 256) {
        const long e = r + j;
        double s = V[e] * (double)GM[e];                 // -V_ij rho_ij
        if (j == i) s += sigma * h;
        const T stv = (T)(s - Sigma0[e]);
        St[e] = stv;
        if (Lm) {
            // end-point matrices of the Fourier route: L = St/2 - dtau (Sc_0 + Sc_M)/4, R = G_0 + G_M
            Lm[e] = T(0.5) * stv - T(0.25) * dtau * (Sc0[e] + ScM[e]);
            Rm[e] = G0[e] + GM[e];
        }
    }
}

// ------------------------------------------------------------ FFT in LDS
// Workgroups are dealt to the 8 XCDs round-robin by block index; renumbered so
// that each XCD takes a contiguous range, neighbouring column groups (which
// share 128-byte lines of every row) run under the same L2 instead of each
// XCD fetching the whole line for its half.
__device__ __forceinline__ long xcd_block(long b, long nb) {
    const long x = b & 7, k = b >> 3;
    return x * (nb >> 3) + (x < (nb & 7) ? x : (nb & 7)) + k;
}

constexpr int FFT_UNR = 8;   // loads of a thread in flight at once when filling LDS

__device__ __forceinline__ int bitrev(int x, int L) { return (int)(__brev((unsigned)x) >> (32 - L)); }

// Decimation-in-time stages over CW bit-reversed columns of M = 2^L points in
// LDS (br, bi), twiddles W_M^j = e^(-2 pi i j / M), j < M/2, in LDS (twr, twi).
// Stages are taken two at a time as radix-4 butterflies (half the LDS passes
// and barriers of radix-2); an odd L starts with one radix-2 stage. For the
// stage pair (s, s+1), h = 2^(s-1), a butterfly takes the points pos, pos+h,
// pos+2h, pos+3h of a group of 4h (pos < h): stage s pairs (pos, pos+h) and
// (pos+2h, pos+3h) with W_2h^pos, stage s+1 pairs (pos, pos+2h) with W_4h^pos
// and (pos+h, pos+3h) with W_4h^(pos+h) = -i W_4h^pos.
template <class T>
__device__ void fft_stages(T* br, T* bi, int M, int L, int CW, const T* __restrict__ twr, const T* __restrict__ twi) {
    int s = 1;
    if (L & 1) {
        for (int b = threadIdx.x; b < (M >> 1) * CW; b += blockDim.x) {
            const int w = b / (M >> 1), bb = b % (M >> 1);
            const int i0 = w * M + 2 * bb, i1 = i0 + 1;
            const T ar = br[i1], ai = bi[i1], ur = br[i0], ui = bi[i0];
            br[i0] = ur + ar;
            bi[i0] = ui + ai;
            br[i1] = ur - ar;
            bi[i1] = ui - ai;
        }
        __syncthreads();
        s = 2;
    }
    for (; s < L; s += 2) {
        const int h = 1 << (s - 1);
        const int st2 = M >> s, st4 = M >> (s + 1);          // twiddle strides of W_2h and W_4h
        for (int b = threadIdx.x; b < (M >> 2) * CW; b += blockDim.x) {
            const int w = b / (M >> 2), bb = b % (M >> 2);
            const int grp = bb >> (s - 1), pos = bb & (h - 1);
            const int i0 = w * M + grp * 4 * h + pos;
            const T a0r = br[i0], a0i = bi[i0], a1r = br[i0 + h], a1i = bi[i0 + h];
            const T a2r = br[i0 + 2 * h], a2i = bi[i0 + 2 * h], a3r = br[i0 + 3 * h], a3i = bi[i0 + 3 * h];
            const T w2r = twr[pos * st2], w2i = twi[pos * st2];
            const T w4r = twr[pos * st4], w4i = twi[pos * st4];
            // stage s
            const T t1r = a1r * w2r - a1i * w2i, t1i = a1r * w2i + a1i * w2r;
            const T t3r = a3r * w2r - a3i * w2i, t3i = a3r * w2i + a3i * w2r;
            const T b0r = a0r + t1r, b0i = a0i + t1i, b1r = a0r - t1r, b1i = a0i - t1i;
            const T b2r = a2r + t3r, b2i = a2i + t3i, b3r = a2r - t3r, b3i = a2i - t3i;
            // stage s + 1: u2 = W_4h^pos b2, u3 = -i W_4h^pos b3
            const T u2r = b2r * w4r - b2i * w4i, u2i = b2r * w4i + b2i * w4r;
            const T v3r = b3r * w4r - b3i * w4i, v3i = b3r * w4i + b3i * w4r;
            const T u3r = v3i, u3i = -v3r;
            br[i0] = b0r + u2r;
            bi[i0] = b0i + u2i;
            br[i0 + 2 * h] = b0r - u2r;
            bi[i0 + 2 * h] = b0i - u2i;
            br[i0 + h] = b1r + u3r;
            bi[i0 + h] = b1i + u3i;
            br[i0 + 3 * h] = b1r - u3r;
            bi[i0 + 3 * h] = b1i - u3i;
        }
        __syncthreads();
    }
}

// Twiddles W_M^j, j < M/2: the global table holds the real parts, then the
// imaginary parts. With lds set they are copied into LDS after the columns
// (twr, twi point there on return); otherwise they are read from the table
// (the largest transforms, whose columns leave no room for them).
template <class T>
__device__ __forceinline__ void fft_twiddles(int M, int lds, const T* __restrict__ tw, T* sm, const T*& twr,
                                             const T*& twi) {
    if (lds) {
        for (int j = threadIdx.x; j < M; j += blockDim.x) sm[j] = tw[j];
        twr = sm;
    } else {
        twr = tw;
    }
    twi = twr + (M >> 1);
}

// A_k = sum_{q<M} x^_q e^(-i pi (2k+1) q / M) for k < M/2 and every real column
// of X [M+1][nc], with x^_0 = (X_0 - X_M)/2. Output planar [M/2][nc], written
// as s A_k + D (s real; D real [nc], nullable, added to every real part).
template <class T>
__global__ __launch_bounds__(1024) void k_fft_fwd(int nc, int M, int L, int CW, int tw_lds, const T* X,
                                                 const T* __restrict__ twist, const T* __restrict__ tw, T osc,
                                                 const T* oadd, T* Are, T* Aim, long nblk1, const T* X2, T* Are2,
                                                 T* Aim2) {
    extern __shared__ unsigned char sm_raw[];
    T* br = reinterpret_cast<T*>(sm_raw);
    T* bi = br + CW * M;
    const T *twr, *twi;
    fft_twiddles(M, tw_lds, tw, bi + CW * M, twr, twi);
    // workgroups from nblk1 on transform a second tensor X2 (plain, into Are2, Aim2)
    long bx = xcd_block(blockIdx.x, gridDim.x);
    if (X2 && bx >= nblk1) {
        bx -= nblk1;
        X = X2;
        Are = Are2;
        Aim = Aim2;
        osc = T(1);
        oadd = nullptr;
    }
    const long c0 = bx * 2 * CW;
    // row q = 0 holds x^_0 = (X_0 - X_M) / 2 (twist factor 1)
    if (threadIdx.x < CW) {
        const int w = threadIdx.x;
        const long c1 = c0 + 2 * w, c2 = c1 + 1;
        const T x1 = c1 < nc ? T(0.5) * (X[c1] - X[(long)M * nc + c1]) : T(0);
        const T x2 = c2 < nc ? T(0.5) * (X[c2] - X[(long)M * nc + c2]) : T(0);
        br[w * M] = x1;
        bi[w * M] = x2;
    }
    // rows q >= 1: FFT_UNR rows of the thread's loads are in flight at once (a
    // plain strided loop waits out one memory latency per row)
    for (int base = CW + threadIdx.x; base < M * CW; base += FFT_UNR * blockDim.x) {
        T x1[FFT_UNR], x2[FFT_UNR];
#pragma unroll
        for (int u = 0; u < FFT_UNR; ++u) {
            const int idx = base + u * blockDim.x;
            const int q = idx / CW, w = idx % CW;
            const long c1 = c0 + 2 * w, c2 = c1 + 1;
            const bool in = idx < M * CW;
            x1[u] = (in && c1 < nc) ? X[(long)q * nc + c1] : T(0);
            x2[u] = (in && c2 < nc) ? X[(long)q * nc + c2] : T(0);
        }
#pragma unroll
        for (int u = 0; u < FFT_UNR; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < M * CW) {
                const int q = idx / CW, w = idx % CW;
                const T cr = twist[2 * q], ci = twist[2 * q + 1];
                const int r = w * M + bitrev(q, L);
                br[r] = x1[u] * cr - x2[u] * ci;
                bi[r] = x1[u] * ci + x2[u] * cr;
            }
        }
    }
    __syncthreads();
    fft_stages(br, bi, M, L, CW, twr, twi);
    for (int idx = threadIdx.x; idx < (M >> 1) * CW; idx += blockDim.x) {
        const int k = idx / CW, w = idx % CW;
        const long c1 = c0 + 2 * w, c2 = c1 + 1;
        const T zr = br[w * M + k], zi = bi[w * M + k];
        const T yr = br[w * M + M - 1 - k], yi = bi[w * M + M - 1 - k];
        if (c1 < nc) {
            Are[(long)k * nc + c1] = osc * (T(0.5) * (zr + yr)) + (oadd ? oadd[c1] : T(0));
            Aim[(long)k * nc + c1] = osc * (T(0.5) * (zi - yi));
        }
        if (c2 < nc) {
            Are[(long)k * nc + c2] = osc * (T(0.5) * (zi + yi)) + (oadd ? oadd[c2] : T(0));
            Aim[(long)k * nc + c2] = osc * (T(-0.5) * (zr - yr));
        }
    }
}

// out_q = (1/M) sum_{k<M} C_k e^(i pi (2k+1) q / M), q < M, for real outputs
// whose spectra satisfy C_(M-1-k) = conj(C_k); input planar [M/2][nc].
template <class T>
__global__ __launch_bounds__(1024) void k_fft_inv(int nc, int M, int L, int CW, int tw_lds, const T* __restrict__ Cre,
                                                 const T* __restrict__ Cim, const T* __restrict__ twist,
                                                 const T* __restrict__ tw, T* __restrict__ out) {
    extern __shared__ unsigned char sm_raw[];
    T* br = reinterpret_cast<T*>(sm_raw);
    T* bi = br + CW * M;
    const T *twr, *twi;
    fft_twiddles(M, tw_lds, tw, bi + CW * M, twr, twi);
    const long c0 = xcd_block(blockIdx.x, gridDim.x) * 2 * CW;
    for (int idx = threadIdx.x; idx < (M >> 1) * CW; idx += blockDim.x) {
        const int k = idx / CW, w = idx % CW;
        const long c1 = c0 + 2 * w, c2 = c1 + 1;
        T a_r = 0, a_i = 0, b_r = 0, b_i = 0;
        if (c1 < nc) { a_r = Cre[(long)k * nc + c1]; a_i = Cim[(long)k * nc + c1]; }
        if (c2 < nc) { b_r = Cre[(long)k * nc + c2]; b_i = Cim[(long)k * nc + c2]; }
        // Z_k = C1_k + i C2_k, Z_(M-1-k) = conj(C1_k) + i conj(C2_k); store conj(Z)
        const int r0 = w * M + bitrev(k, L), r1 = w * M + bitrev(M - 1 - k, L);
        br[r0] = a_r - b_i;
        bi[r0] = -(a_i + b_r);
        br[r1] = a_r + b_i;
        bi[r1] = -(b_r - a_i);
    }
    __syncthreads();
    fft_stages(br, bi, M, L, CW, twr, twi);
    const T sc = T(1) / T(M);
    for (int idx = threadIdx.x; idx < M * CW; idx += blockDim.x) {
        const int q = idx / CW, w = idx % CW;
        const long c1 = c0 + 2 * w, c2 = c1 + 1;
        const T yr = br[w * M + q] * sc, yi = -bi[w * M + q] * sc;
        const T cr = twist[2 * q], ci = twist[2 * q + 1];          // e^(-i pi q/M); multiply by its conjugate
        if (c1 < nc) out[(long)q * nc + c1] = yr * cr + yi * ci;
        if (c2 < nc) out[(long)q * nc + c2] = yi * cr - yr * ci;
    }
}

// I1_0 += E, I1_M = St R - I1_0
template <class T>
__global__ void k_endpoint_final(long nn, const T* E, const T* SR, T* I0, T* IM) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
        const T v = I0[e] + E[e];
        I0[e] = v;
        IM[e] = SR[e] - v;
    }
}

// ------------------------------------------------------------ direct quadrature (any grid)
struct Stencil {
    int cnt;
    int node[8];
    double wt[8];
};

__device__ void interp4(const double* tau, int n_tau, int block, double s, double scale, Stencil& st) {
    int lo = 0, hi = n_tau - 1;                    // largest a with tau[a] <= s
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tau[mid] <= s) lo = mid;
        else hi = mid;
    }
    int a = tau[hi] <= s ? hi : lo;
    if (a > n_tau - 2) a = n_tau - 2;
    if (a < 0) a = 0;
    const int blo = (a / block) * block;
    const int bhi = min(blo + block, n_tau - 1);
    int start = a - 1;
    if (start < blo) start = blo;
    if (start > bhi - 3) start = bhi - 3;
    for (int m = 0; m < 4; ++m) {
        double w = 1.0;
        for (int j = 0; j < 4; ++j)
            if (j != m) w *= (s - tau[start + j]) / (tau[start + m] - tau[start + j]);
        st.node[st.cnt] = start + m;
        st.wt[st.cnt] = scale * w;
        ++st.cnt;
    }
}

__device__ void make_stencil(int p, int q, int n_tau, int kind, int block, const double* tau,
                             const double* w, Stencil& st) {
    const int M = n_tau - 1;
    const double beta = tau[M];
    st.cnt = 0;
    if (p > 0 && q <= p) {
        const double wl = q < p ? w[q] : 0.5 * (tau[p] - tau[p - 1]);
        if (q == p) { st.node[st.cnt] = 0; st.wt[st.cnt++] = wl; }
        else if (kind == NEGF_TAU_UNIFORM) { st.node[st.cnt] = p - q; st.wt[st.cnt++] = wl; }
        else interp4(tau, n_tau, block, tau[p] - tau[q], wl, st);
    }
    if (p < M && q >= p) {
        const double wr = q > p ? w[q] : 0.5 * (tau[p + 1] - tau[p]);
        if (q == p) { st.node[st.cnt] = M; st.wt[st.cnt++] = -wr; }
        else if (kind == NEGF_TAU_UNIFORM) { st.node[st.cnt] = M + p - q; st.wt[st.cnt++] = -wr; }
        else interp4(tau, n_tau, block, beta + tau[p] - tau[q], -wr, st);
    }
}

// Out[p] = sum_q sum_m wt_m Sc[node_m] G[q] for a strip of 64 rows of slice p and
// up to 2 x JTW x 16 columns starting at c0. The interpolated Sigma_c rows (the A
// operand) are formed once per (p, q, k-panel) and used against the whole strip
// of columns, so the kernel is bound by the matrix cores rather than by the
// reads of the interpolation nodes. 8 waves: wave w owns row tile w & 3 and the
// column tiles (w >> 2) + 2 t. Stencils of 32 values of q are built at a time.
template <class T, int JTW>
__global__ __launch_bounds__(512) void k_conv_strip(int n, int n_tau, int kind, int block,
                                                    const double* __restrict__ tau, const double* __restrict__ w,
                                                    const T* __restrict__ Sc, const T* __restrict__ G,
                                                    T* __restrict__ Out, int c0, int c1) {
    constexpr int BK = 16, CWP = 2 * JTW * 16;
    __shared__ T As[BK][65];
    __shared__ T Bs[BK][CWP + 1];
    __shared__ Stencil sst[32];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rt = wv & 3, cg = wv >> 2;
    // XCD-aware order: each XCD takes a contiguous range of (p, strip) so that the
    // blocks resident on it share the G panels and nearby Sigma_c nodes in its L2
    const int nstrip = (n + 63) / 64;
    const long nblk = (long)gridDim.x;
    const long xb = blockIdx.x & 7, kb = blockIdx.x >> 3;
    const long lb = xb * (nblk >> 3) + (xb < (nblk & 7) ? xb : (nblk & 7)) + kb;
    const int p = (int)(lb / nstrip), m0 = (int)(lb % nstrip) * 64;
    const long nn = (long)n * n;
    typename Mma<T>::acc_t acc[JTW];
#pragma unroll
    for (int t = 0; t < JTW; ++t) acc[t] = Mma<T>::zero();
    for (int q0 = 0; q0 < n_tau; q0 += 32) {
        __syncthreads();
        if (tid < 32) {
            if (q0 + tid < n_tau) make_stencil(p, q0 + tid, n_tau, kind, block, tau, w, sst[tid]);
            else sst[tid].cnt = 0;
        }
        __syncthreads();
        const int qn = min(32, n_tau - q0);
        for (int qq = 0; qq < qn; ++qq) {
            const int cnt = sst[qq].cnt;
            if (cnt == 0) continue;
            const T* Gq = G + (long)(q0 + qq) * nn;
            for (int k0 = 0; k0 < n; k0 += BK) {
                for (int e = tid; e < 64 * BK; e += 512) {
                    const int m = e / BK, kk = e - m * BK;
                    const int row = m0 + m, k = k0 + kk;
                    double v = 0.0;
                    if (row < n && k < n)
                        for (int c = 0; c < cnt; ++c)
                            v += sst[qq].wt[c] * (double)Sc[(long)sst[qq].node[c] * nn + (long)row * n + k];
                    As[kk][m] = (T)v;
                }
                for (int e = tid; e < BK * CWP; e += 512) {
                    const int kk = e / CWP, j = e - kk * CWP;
                    const int k = k0 + kk, col = c0 + j;
                    Bs[kk][j] = (k < n && col < c1) ? Gq[(long)k * n + col] : T(0);
                }
                __syncthreads();
#pragma unroll
                for (int ks = 0; ks < BK / 4; ++ks) {
                    const int kk = ks * 4 + (lane >> 4);
                    AFrag<T> a;
                    a.load(lane, [&](int m) { return As[kk][rt * 16 + m]; });
#pragma unroll
                    for (int t = 0; t < JTW; ++t) acc[t] = a.mma(Bs[kk][(cg + 2 * t) * 16 + (lane & 15)], acc[t]);
                }
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int t = 0; t < JTW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + rt * 16 + Mma<T>::row(lane, r);
            const int col = c0 + (cg + 2 * t) * 16 + (lane & 15);
            if (row < n && col < c1) Out[(long)p * nn + (long)row * n + col] = acc[t][r];
        }
}

template <class T>
int conv_strip_launch(int n, int n_tau, int kind, int block, const double* tau, const double* w, const T* Sc,
                      const T* G, T* Out, hipStream_t st) {
    const int ct = (n + 15) / 16;                 // column tiles
    const int jtw = (ct + 1) / 2;

    const dim3 grid((unsigned)(((n + 63) / 64) * n_tau));
    auto go = [&](auto jt_const) -> int {
        constexpr int JT = decltype(jt_const)::value;
        for (int c0 = 0; c0 < n; c0 += 2 * JT * 16) {
            const int c1 = min(n, c0 + 2 * JT * 16);
            hipLaunchKernelGGL((k_conv_strip<T, JT>), grid, dim3(512), 0, st, n, n_tau, kind, block, tau, w, Sc, G,
                               Out, c0, c1);
            LAUNCH_CHECK();
        }
        return NEGF_OK;
    };
    if (jtw <= 2) return go(std::integral_constant<int, 2>());
    if (jtw <= 4) return go(std::integral_constant<int, 4>());
    if (jtw <= 7) return go(std::integral_constant<int, 7>());
    return go(std::integral_constant<int, 13>());
}

// ------------------------------------------------------------ eigenbasis recurrences
// Ea[k][q] = e^(-a tau_q), Eb[k][q] = e^(-a (beta - tau_q)), dec[k][q] = e^(-a (tau_(q+1) - tau_q)),
// a = |eps_k - mu|; cpre[k] = 1 / (1 + e^(-a beta)). The tables are k-major: the
// recurrences of one workgroup share one or two values of k and walk q, so
// their table reads are contiguous runs instead of one value per cache line.
__global__ void k_scan_tables(int n, int n_tau, const double* __restrict__ tau, double beta,
                              const double* __restrict__ eps, double mu, double* Ea, double* Eb, double* dec,
                              double* cpre) {
    const long tot = (long)n * n_tau;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int k = (int)(e / n_tau), q = (int)(e % n_tau);
        const double a = fabs(eps[k] - mu);
        Ea[e] = exp(-a * tau[q]);
        Eb[e] = exp(-a * (beta - tau[q]));
        dec[e] = q + 1 < n_tau ? exp(-a * (tau[q + 1] - tau[q])) : 0.0;
        if (q == 0) cpre[k] = 1.0 / (1.0 + exp(-a * beta));
    }
}

// Out[p][k][j] = Q_p[-g_k, In[.][k][j]] - g_k(tau_p) C[j][k]: the eigenbasis form
// of G0 + Q[G0, I1] before the final rotation by C, as a forward and a backward
// recurrence over tau per element (k, j). The tau axis is cut into 16 chunks and
// a workgroup holds 16 elements x 16 chunks: each chunk first runs its recurrence
// from zero to get its affine aggregate (acc_out = d acc_in + a), the aggregates
// are folded in LDS to give every chunk its starting value, and the chunk then
// runs again writing the outputs.
template <class T>
__global__ __launch_bounds__(256) void k_eig_scan_chunked(int n, int n_tau, const T* __restrict__ In, T* __restrict__ Out,
                                                          const double* __restrict__ w, const double* __restrict__ hL,
                                                          const double* __restrict__ hR, const double* __restrict__ Ea,
                                                          const double* __restrict__ Eb, const double* __restrict__ dec,
                                                          const double* __restrict__ cpre,
                                                          const double* __restrict__ eps, double mu,
                                                          const double* __restrict__ C) {
    constexpr int NCH = 16, NE = 16;
    __shared__ double sd[NCH][NE + 1], sa[NCH][NE + 1];
    const int el = threadIdx.x & (NE - 1), ch = threadIdx.x / NE;
    const long nn = (long)n * n;
    const long e = xcd_block(blockIdx.x, gridDim.x) * NE + el;   // XCD-contiguous, as in the transforms
    const bool ok = e < nn;
    const int k = ok ? (int)(e / n) : 0, j = ok ? (int)(e % n) : 0;
    const bool pos = ok && eps[k] - mu >= 0.0;
    const long tk = (long)k * n_tau;                 // row k of the k-major tables
    const double c = ok ? cpre[k] : 0.0;
    const int M = n_tau - 1, P = n_tau;
    const int p0 = (int)((long)ch * P / NCH), p1 = (int)((long)(ch + 1) * P / NCH);
    auto fold_fwd = [&](double& start) {
        start = 0.0;
        for (int cc = 0; cc < ch; ++cc) start = sd[cc][el] * start + sa[cc][el];
    };
    auto fold_bwd = [&](double& start) {
        start = 0.0;
        for (int cc = NCH - 1; cc > ch; --cc) start = sd[cc][el] * start + sa[cc][el];
    };
    // ---- forward recurrence (lower part of the convolution)
    {
        double acc = 0.0, d = 1.0;
        if (ok) {
            for (int p = p0; p < p1; ++p) {
                const double b = (double)In[(long)p * nn + e];
                if (pos) {
                    if (p < M) {
                        const double dp = dec[tk + p];
                        acc = dp * (acc + w[p] * b);
                        d *= dp;
                    }
                } else {
                    acc += w[p] * Ea[tk + p] * b;
                }
            }
        }
        sd[ch][el] = d;
        sa[ch][el] = acc;
        __syncthreads();
        fold_fwd(acc);
        if (ok) {
            for (int p = p0; p < p1; ++p) {
                const double b = (double)In[(long)p * nn + e];
                if (pos) {
                    Out[(long)p * nn + e] = (T)(c * (acc + hL[p] * b));
                    if (p < M) acc = dec[tk + p] * (acc + w[p] * b);
                } else {
                    const double ea = Ea[tk + p];
                    Out[(long)p * nn + e] = (T)(c * Eb[tk + p] * (acc + hL[p] * ea * b));
                    acc += w[p] * ea * b;
                }
            }
        }
        __syncthreads();
    }
    // ---- backward recurrence (upper part), combined with the forward result
    {
        double acc = 0.0, d = 1.0;
        if (ok) {
            for (int p = p1 - 1; p >= p0; --p) {
                const double b = (double)In[(long)p * nn + e];
                if (pos) {
                    acc += w[p] * Eb[tk + p] * b;
                } else if (p > 0) {
                    const double dp = dec[tk + p - 1];
                    acc = dp * (acc + w[p] * b);
                    d *= dp;
                }
            }
        }
        sd[ch][el] = d;
        sa[ch][el] = acc;
        __syncthreads();
        fold_bwd(acc);
        if (ok) {
            const double cjk = C[(long)j * n + k];
            for (int p = p1 - 1; p >= p0; --p) {
                const double b = (double)In[(long)p * nn + e];
                const double L = (double)Out[(long)p * nn + e];
                if (pos) {
                    const double eb = Eb[tk + p], ea = Ea[tk + p];
                    const double R = c * ea * (acc + hR[p] * eb * b);
                    acc += w[p] * eb * b;
                    Out[(long)p * nn + e] = (T)(-L + R - c * ea * cjk);
                } else {
                    const double R = c * (acc + hR[p] * b);
                    if (p > 0) acc = dec[tk + p - 1] * (acc + w[p] * b);
                    Out[(long)p * nn + e] = (T)(-L + R - c * Eb[tk + p] * cjk);
                }
            }
        }
    }
}

// The same recurrences with In read once and Out written once: the tau axis is
// cut into 32 chunks of at most CL points, a workgroup holds 16 elements x 32
// chunks, and each thread keeps its chunk of In and of the forward results in
// registers. Both aggregates (forward and backward) come from one pass over the
// registers, are folded in LDS, and the forward and backward output sweeps run
// over the registers; only the final values are stored. Needs n_tau <= 32 CL.
//
// With TL the workgroup first copies the table rows of its values of k (at most
// two, since its 16 consecutive elements (k, j) span at most two rows when
// n >= 16) into LDS, so the recurrences read them there instead of from the L2.
template <class T, int CL, bool TL>
__global__ __launch_bounds__(512) void k_eig_scan_reg(int n, int n_tau, const T* __restrict__ In, T* __restrict__ Out,
                                                      const double* __restrict__ w, const double* __restrict__ hL,
                                                      const double* __restrict__ hR, const double* __restrict__ Ea_g,
                                                      const double* __restrict__ Eb_g, const double* __restrict__ dec_g,
                                                      const double* __restrict__ cpre,
                                                      const double* __restrict__ eps, double mu,
                                                      const double* __restrict__ C) {
    constexpr int NCH = 32, NE = 16;
    __shared__ double sdf[NCH][NE + 1], saf[NCH][NE + 1], sdb[NCH][NE + 1], sab[NCH][NE + 1];
    extern __shared__ double tsm[];                  // TL: [2 rows][Ea, Eb, dec][n_tau]
    const int el = threadIdx.x & (NE - 1), ch = threadIdx.x / NE;
    const long nn = (long)n * n;
    const long e = xcd_block(blockIdx.x, gridDim.x) * NE + el;   // XCD-contiguous, as in the transforms
    const bool ok = e < nn;
    const int k = ok ? (int)(e / n) : 0, j = ok ? (int)(e % n) : 0;
    const bool pos = ok && eps[k] - mu >= 0.0;
    const double c = ok ? cpre[k] : 0.0;
    const int M = n_tau - 1, P = n_tau;
    const int p0 = (int)((long)ch * P / NCH), p1 = (int)((long)(ch + 1) * P / NCH);
    double b[CL], L[CL];
#pragma unroll
    for (int t = 0; t < CL; ++t) b[t] = (ok && p0 + t < p1) ? (double)In[(long)(p0 + t) * nn + e] : 0.0;
    const double *Ea, *Eb, *dec;
    long tk;                                         // offset of row k in the tables read
    if constexpr (TL) {
        const long e0 = xcd_block(blockIdx.x, gridDim.x) * NE;
        const int k0 = (int)(e0 / n), k1 = (int)((e0 + NE - 1 < nn ? e0 + NE - 1 : nn - 1) / n);
        for (int r = 0; r <= k1 - k0; ++r)
            for (int q = threadIdx.x; q < n_tau; q += 512) {
                const long g = (long)(k0 + r) * n_tau + q;
                tsm[(3 * r + 0) * n_tau + q] = Ea_g[g];
                tsm[(3 * r + 1) * n_tau + q] = Eb_g[g];
                tsm[(3 * r + 2) * n_tau + q] = dec_g[g];
            }
        __syncthreads();
        const double* row = tsm + 3 * (ok ? k - k0 : 0) * n_tau;
        Ea = row;
        Eb = row + n_tau;
        dec = row + 2 * n_tau;
        tk = 0;
    } else {
        Ea = Ea_g;
        Eb = Eb_g;
        dec = dec_g;
        tk = (long)k * n_tau;                        // row k of the k-major tables
    }
    // chunk aggregates: acc_out = d acc_in + a, forward (increasing p) and backward
    {
        double af = 0.0, df = 1.0, ab = 0.0, db = 1.0;
        if (ok) {
#pragma unroll
            for (int t = 0; t < CL; ++t) {
                const int p = p0 + t;
                if (p < p1) {
                    if (pos) {
                        if (p < M) {
                            const double dp = dec[tk + p];
                            af = dp * (af + w[p] * b[t]);
                            df *= dp;
                        }
                    } else {
                        af += w[p] * Ea[tk + p] * b[t];
                    }
                }
            }
#pragma unroll
            for (int t = CL - 1; t >= 0; --t) {
                const int p = p0 + t;
                if (p < p1) {
                    if (pos) {
                        ab += w[p] * Eb[tk + p] * b[t];
                    } else if (p > 0) {
                        const double dp = dec[tk + p - 1];
                        ab = dp * (ab + w[p] * b[t]);
                        db *= dp;
                    }
                }
            }
        }
        sdf[ch][el] = df;
        saf[ch][el] = af;
        sdb[ch][el] = db;
        sab[ch][el] = ab;
    }
    __syncthreads();
    if (!ok) return;
    // forward sweep (lower part of the convolution)
    {
        double acc = 0.0;
        for (int cc = 0; cc < ch; ++cc) acc = sdf[cc][el] * acc + saf[cc][el];
#pragma unroll
        for (int t = 0; t < CL; ++t) {
            const int p = p0 + t;
            if (p < p1) {
                if (pos) {
                    L[t] = c * (acc + hL[p] * b[t]);
                    if (p < M) acc = dec[tk + p] * (acc + w[p] * b[t]);
                } else {
                    const double ea = Ea[tk + p];
                    L[t] = c * Eb[tk + p] * (acc + hL[p] * ea * b[t]);
                    acc += w[p] * ea * b[t];
                }
            }
        }
    }
    // backward sweep (upper part), combined with the forward result
    {
        double acc = 0.0;
        for (int cc = NCH - 1; cc > ch; --cc) acc = sdb[cc][el] * acc + sab[cc][el];
        const double cjk = C[(long)j * n + k];
#pragma unroll
        for (int t = CL - 1; t >= 0; --t) {
            const int p = p0 + t;
            if (p < p1) {
                if (pos) {
                    const double eb = Eb[tk + p], ea = Ea[tk + p];
                    const double R = c * ea * (acc + hR[p] * eb * b[t]);
                    acc += w[p] * eb * b[t];
                    Out[(long)p * nn + e] = (T)(-L[t] + R - c * ea * cjk);
                } else {
                    const double R = c * (acc + hR[p] * b[t]);
                    if (p > 0) acc = dec[tk + p - 1] * (acc + w[p] * b[t]);
                    Out[(long)p * nn + e] = (T)(-L[t] + R - c * Eb[tk + p] * cjk);
                }
            }
        }
    }
}

// G[s] <- (G[s] + G[s]^T)/2 for every slice, by pairs of 32 x 32 tiles (I, J),
// I <= J: both tiles are read row-wise into LDS and written back row-wise.
// grid.x = tile pair, grid.y = slice.
template <class T>
__global__ __launch_bounds__(256) void k_symmetrize(int n, int nt, int npair, T* G) {
    __shared__ T A[32][33], B[32][33];
    // one workgroup per (slice, tile pair), XCD-contiguous so that the tiles of a
    // slice, which share the lines at their edges, run under one L2; tile pair
    // index -> (I, J), I <= J, row-major over the upper triangle of tiles
    const long lbk = xcd_block(blockIdx.x, gridDim.x);
    const long sl = lbk / npair;
    int r = (int)(lbk - sl * npair), I = 0;
    while (r >= nt - I) {
        r -= nt - I;
        ++I;
    }
    const int J = I + r;
    T* g = G + sl * n * n;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int yy = ty; yy < 32; yy += 8) {
        const int ra = I * 32 + yy, ca = J * 32 + tx;
        A[yy][tx] = (ra < n && ca < n) ? g[(long)ra * n + ca] : T(0);
        const int rb = J * 32 + yy, cb = I * 32 + tx;
        B[yy][tx] = (rb < n && cb < n) ? g[(long)rb * n + cb] : T(0);
    }
    __syncthreads();
    for (int yy = ty; yy < 32; yy += 8) {
        const int ra = I * 32 + yy, ca = J * 32 + tx;
        if (ra < n && ca < n) g[(long)ra * n + ca] = T(0.5) * (A[yy][tx] + B[tx][yy]);
        const int rb = J * 32 + yy, cb = I * 32 + tx;
        if (I != J && rb < n && cb < n) g[(long)rb * n + cb] = T(0.5) * (B[yy][tx] + A[tx][yy]);
    }
}

// ------------------------------------------------------------ energy
// part[q][I] = sum over rows i of strip I (32 rows) of sum_j S_ij G_ji with
// S = Sc(beta - tau_q), G = G(tau_q): float64 products, compensated sums kept
// as unrounded (sum, compensation) pairs. One
// workgroup per (q, I); G is read through LDS one 32 x 32 block at a time, so
// that both S (block (I, J)) and G (block (J, I)) are read along their rows,
// and a thread's loads for EN_MAXJ blocks of the strip are issued before the
// first of them is summed. Tr[Sc(beta - tau_q) G(tau_q)] = sum_I part[q][I].
constexpr int EN_MAXJ = 4;                             // blocks of a strip whose loads are in flight together
template <class T>
__global__ __launch_bounds__(256) void k_energy_slices(int n, int n_tau, int nI, const T* __restrict__ Sc,
                                                       const T* __restrict__ G, double* part) {
    __shared__ double red[2 * (256 / 64) + 2];
    __shared__ double gt[32][33];
    // XCD-contiguous: the strips of a slice read G at neighbouring columns of
    // every row, and run under one L2
    const long lbk = xcd_block(blockIdx.x, gridDim.x);
    const int q = (int)(lbk / nI), yb = (int)(lbk - (long)q * nI), I = 32 * yb;
    const long nn = (long)n * n;
    const T* S = Sc + (long)(n_tau - 1 - q) * nn;
    const T* g = G + (long)q * nn;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;     // 32 x 8 threads
    const int nJ = (n + 31) >> 5;
    CSum s{0.0, 0.0};
    for (int J0 = 0; J0 < nJ; J0 += EN_MAXJ) {
        double gv[EN_MAXJ][4], sv[EN_MAXJ][4];
#pragma unroll
        for (int jj = 0; jj < EN_MAXJ; ++jj)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int J = 32 * (J0 + jj), r = ty + 8 * u;
                const bool inb = J0 + jj < nJ;
                // gv: G[J + r][I + tx] (row r of block (J, I)); sv: S[I + r][J + tx]
                gv[jj][u] = (inb && J + r < n && I + tx < n) ? (double)g[(long)(J + r) * n + I + tx] : 0.0;
                sv[jj][u] = (inb && I + r < n && J + tx < n) ? (double)S[(long)(I + r) * n + J + tx] : 0.0;
            }
#pragma unroll
        for (int jj = 0; jj < EN_MAXJ; ++jj) {
            if (J0 + jj < nJ) {
                __syncthreads();
#pragma unroll
                for (int u = 0; u < 4; ++u) gt[tx][ty + 8 * u] = gv[jj][u];      // gt[c][r] = G[J + r][I + c]
                __syncthreads();
                // S[I + r][J + c] * G[J + c][I + r], G from gt[r][c]
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int r = ty + 8 * u;
                    if (I + r < n && 32 * (J0 + jj) + tx < n) s.add(sv[jj][u] * gt[r][tx]);
                }
            }
        }
    }
    const CSum tot = block_csum_pair<256>(s, red);
    if (threadIdx.x == 0) {
        part[2 * ((long)q * nI + yb)] = tot.s;
        part[2 * ((long)q * nI + yb) + 1] = tot.c;
    }
}

// Static part per row i of rho = -G(beta^-): rowpart[i] = (sum_j h_ij rho_ji,
// sum_j [sigma rho_ii V_ij rho_jj - V_ij rho_ij rho_ji], rho_ii), one workgroup
// per row, compensated sums in a fixed order kept as (sum, compensation) pairs.
template <class T>
__global__ __launch_bounds__(256) void k_energy_rows(int n, int sigma, const double* __restrict__ h,
                                                     const double* __restrict__ V, const T* __restrict__ GM,
                                                     double* __restrict__ rowpart) {
    __shared__ double red[2 * (256 / 64) + 2];
    const int i = blockIdx.x;
    const double rii = -(double)GM[(long)i * n + i];
    CSum c1{0.0, 0.0}, c2{0.0, 0.0};
    for (int j = threadIdx.x; j < n; j += 256) {
        const long e = (long)i * n + j;
        const double rij = -(double)GM[e], rji = -(double)GM[(long)j * n + i];
        const double rjj = -(double)GM[(long)j * n + j];
        c1.add(h[e] * rji);
        c2.add(sigma * rii * V[e] * rjj);
        c2.add(-(V[e] * rij * rji));
    }
    const CSum e1 = block_csum_pair<256>(c1, red);
    const CSum e2 = block_csum_pair<256>(c2, red);
    if (threadIdx.x == 0) {
        rowpart[5 * i] = e1.s;
        rowpart[5 * i + 1] = e1.c;
        rowpart[5 * i + 2] = e2.s;
        rowpart[5 * i + 3] = e2.c;
        rowpart[5 * i + 4] = rii;
    }
}

// E = sigma (sum_ij h_ij rho_ji + (1/2) [Hartree - exchange]) - (sigma/2) sum_q w_q part[q];
// N = sigma Tr rho. One workgroup over the slice and row partials.
__global__ __launch_bounds__(256) void k_energy_final(int n, int n_tau, int sigma, const double* __restrict__ w,
                                                      const double* __restrict__ part,
                                                      const double* __restrict__ rowpart, double* out) {
    __shared__ double red[2 * (256 / 64) + 2];
    const int nI = (n + 31) >> 5;
    CSum cec{0.0, 0.0};
    for (int q = threadIdx.x; q < n_tau; q += 256) {
        CSum tq{0.0, 0.0};                                 // Tr[Sc(beta - tau_q) G(tau_q)], strips in order
        for (int I = 0; I < nI; ++I) tq.merge(part[2 * ((long)q * nI + I)], part[2 * ((long)q * nI + I) + 1]);
        cec.add(w[q] * tq.value());
    }
    const double ec = block_csum<256>(cec, red);
    CSum c1{0.0, 0.0}, c2{0.0, 0.0}, ctr{0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += 256) {
        c1.merge(rowpart[5 * i], rowpart[5 * i + 1]);
        c2.merge(rowpart[5 * i + 2], rowpart[5 * i + 3]);
        ctr.add(rowpart[5 * i + 4]);
    }
    const double e1 = block_csum<256>(c1, red);
    const double e2 = block_csum<256>(c2, red);
    const double tr = block_csum<256>(ctr, red);
    if (threadIdx.x == 0) {
        out[0] = sigma * (e1 + 0.5 * e2) - 0.5 * sigma * ec;
        out[1] = sigma * tr;
    }
}

// ------------------------------------------------------------ density at the nodes
template <class T>
__global__ __launch_bounds__(256) void k_density(int n, int sigma, const double* __restrict__ W,
                                                 const T* __restrict__ GM, double* __restrict__ out) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a < n) out[a] = -sigma * (double)GM[(long)a * n + a] / W[a];
}

// ------------------------------------------------------------ host helpers
void grid_tables(const negf_tau_grid_t* tg, std::vector<double>& w, std::vector<double>& hL,
                 std::vector<double>& hR) {
    const int n = tg->n_tau;
    w.assign(n, 0.0);
    hL.assign(n, 0.0);
    hR.assign(n, 0.0);
    for (int q = 0; q + 1 < n; ++q) {
        const double h = tg->tau[q + 1] - tg->tau[q];
        w[q] += 0.5 * h;
        w[q + 1] += 0.5 * h;
        hR[q] = 0.5 * h;
        hL[q + 1] = 0.5 * h;
    }
}

template <class T>
int fft_tables(negf_ctx* ctx, int M, hipStream_t st, T** twist, T** tw) {
    const std::string tag = std::string(sizeof(T) == 8 ? "fft_d_" : "fft_f_") + std::to_string(M);
    void* p1 = nullptr;
    void* p2 = nullptr;
    if (!ctx->filled[tag]) {
        std::vector<T> a(2 * M), b(M);
        for (int q = 0; q < M; ++q) {
            const long double th = -3.14159265358979323846264338327950288L * q / M;
            a[2 * q] = (T)cosl(th);
            a[2 * q + 1] = (T)sinl(th);
        }
        for (int k = 0; k < M / 2; ++k) {                  // real parts, then imaginary parts
            const long double th = -2.0L * 3.14159265358979323846264338327950288L * k / M;
            b[k] = (T)cosl(th);
            b[M / 2 + k] = (T)sinl(th);
        }
        NEGF_TRY(upload(ctx, (tag + "_twist").c_str(), a.data(), sizeof(T) * a.size(), st, &p1));
        NEGF_TRY(upload(ctx, (tag + "_tw").c_str(), b.data(), sizeof(T) * b.size(), st, &p2));
        ctx->filled[tag] = 1;
    } else {
        NEGF_TRY(scratch(ctx, (tag + "_twist").c_str(), sizeof(T) * 2 * M, &p1));
        NEGF_TRY(scratch(ctx, (tag + "_tw").c_str(), sizeof(T) * M, &p2));
    }
    *twist = (T*)p1;
    *tw = (T*)p2;
    return NEGF_OK;
}

template <class T>
int fft_launch(bool inverse, int nc, int M, const T* in0, const T* in1, T* out0, T* out1, const T* twist,
               const T* tw, hipStream_t st, T oscale = T(1), const T* oadd = nullptr, const T* in0b = nullptr,
               T* out0b = nullptr, T* out1b = nullptr) {
    int L = 0;
    while ((1 << L) < M) ++L;
    // 64 KB of LDS for the columns of a workgroup (8 real columns in float64 at
    // M = 1024, 16 in float32), so that two workgroups share a compute unit and
    // one's loads and stores overlap the other's LDS stages (one workgroup of
    // 16 columns per CU measured 0.15 ms slower per Dyson step at n_b = 199)
    int CW = (int)(65536 / ((long)M * 2 * sizeof(T)));
    if (CW < 1) CW = 1;
    if (CW > 32) CW = 32;
    // the twiddles (M/2 complex) go into LDS after the columns where they fit
    const int tw_lds = ((size_t)CW * M * 2 + (size_t)M) * sizeof(T) <= 160 * 1024 ? 1 : 0;
    const size_t smem = ((size_t)CW * M * 2 + (tw_lds ? (size_t)M : 0)) * sizeof(T);
    const long blocks = ((long)nc + 2 * CW - 1) / (2 * CW);
    const int threads = CW * M >= 4096 ? 1024 : 256;
    static bool attr[2][2] = {{false, false}, {false, false}};
    const int ti = sizeof(T) == 8 ? 0 : 1;
    if (!attr[ti][inverse]) {
        if (inverse) HIP_TRY(hipFuncSetAttribute((const void*)k_fft_inv<T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        else HIP_TRY(hipFuncSetAttribute((const void*)k_fft_fwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        attr[ti][inverse] = true;
    }
    if (!inverse)
        hipLaunchKernelGGL((k_fft_fwd<T>), dim3((unsigned)(in0b ? 2 * blocks : blocks)), dim3(threads), smem, st, nc, M,
                           L, CW, tw_lds, in0, twist, tw, oscale, oadd, out0, out1, blocks, in0b, out0b, out1b);
    else
        hipLaunchKernelGGL((k_fft_inv<T>), dim3((unsigned)blocks), dim3(threads), smem, st, nc, M, L, CW, tw_lds, in0, in1,
                           twist, tw, out0);
    LAUNCH_CHECK();
    return NEGF_OK;
}

}  // namespace

// ============================================================== Dyson step
template <class T>
int dyson_run(negf_ctx* ctx, const negf_tau_grid_t* tg, int n, int sigma, const double* h, const double* V,
              const double* eps, const double* C, double mu, const double* Sigma0, const T* G_in, const T* Sc,
              double alpha, int symmetrize, int conv_algo, T* G_out, hipStream_t st) {
    (void)h;
    const int n_tau = tg->n_tau, M = n_tau - 1;
    const long nn = (long)n * n;
    const bool pow2 = (M & (M - 1)) == 0 && M <= 8192;
    bool use_fft = conv_algo == NEGF_CONV_FFT ||
                   (conv_algo == NEGF_CONV_AUTO && tg->kind == NEGF_TAU_UNIFORM && pow2);
    const double dtau = tg->beta / M;

    std::vector<double> w, hL, hR;
    grid_tables(tg, w, hL, hR);
    std::vector<double> tabs(4 * (size_t)n_tau);
    for (int q = 0; q < n_tau; ++q) {
        tabs[q] = tg->tau[q];
        tabs[n_tau + q] = w[q];
        tabs[2 * n_tau + q] = hL[q];
        tabs[3 * n_tau + q] = hR[q];
    }
    void* dtab = nullptr;
    NEGF_TRY(upload_cached(ctx, "dy_grid", tabs.data(), sizeof(double) * tabs.size(), st, &dtab));
    const double* d_tau = (const double*)dtab;
    const double* d_w = d_tau + n_tau;
    const double* d_hL = d_tau + 2 * n_tau;
    const double* d_hR = d_tau + 3 * n_tau;

    // LS = [Lm | St] and ER = [Em | SR]: the two end-point products L R and St R in one batched launch
    T *LS, *ER, *Rm, *I1, *It;
    NEGF_TRY(scratch_t(ctx, "dy_LS", 2 * nn, &LS));
    NEGF_TRY(scratch_t(ctx, "dy_ER", 2 * nn, &ER));
    NEGF_TRY(scratch_t(ctx, "dy_Rm", nn, &Rm));
    NEGF_TRY(scratch_t(ctx, "dy_I1", nn * n_tau, &I1));
    NEGF_TRY(scratch_t(ctx, "dy_It", nn * n_tau, &It));
    T* const St = LS + nn;
    hipLaunchKernelGGL((k_sigma_tilde<T>), dim3((unsigned)std::max(n, 1)), dim3(256), 0, st, n, sigma, V,
                       G_in + (long)M * nn, Sigma0, St, (T)dtau, Sc, Sc + (long)M * nn, G_in,
                       use_fft ? LS : nullptr, Rm);
    LAUNCH_CHECK();

    // ---------------- I1 = St G + Q[Sigma_c, G]
    if (use_fft) {
        const int nk = M / 2;
        T *Are, *Aim, *Bre, *Bim, *Cre, *Cim, *twist, *tw;
        NEGF_TRY(scratch_t(ctx, "dy_Are", nn * nk, &Are));
        NEGF_TRY(scratch_t(ctx, "dy_Aim", nn * nk, &Aim));
        NEGF_TRY(scratch_t(ctx, "dy_Bre", nn * nk, &Bre));
        NEGF_TRY(scratch_t(ctx, "dy_Bim", nn * nk, &Bim));
        NEGF_TRY(scratch_t(ctx, "dy_Cre", nn * nk, &Cre));
        NEGF_TRY(scratch_t(ctx, "dy_Cim", nn * nk, &Cim));
        NEGF_TRY(fft_tables<T>(ctx, M, st, &twist, &tw));
        // A'_k = dtau A_k + St (St real, the same for every frequency), formed as the transform writes A_k;
        // the transform of G in the same launch
        NEGF_TRY(fft_launch<T>(false, (int)nn, M, Sc, nullptr, Are, Aim, twist, tw, st, (T)dtau, St, G_in, Bre, Bim));
        NEGF_TRY(cgemm<T>(st, n, Are, Aim, Bre, Bim, Cre, Cim, nn, nk));
        NEGF_TRY(fft_launch<T>(true, (int)nn, M, Cre, Cim, I1, nullptr, twist, tw, st));
        // end points p = 0 and p = M: Em = L R, SR = St R
        NEGF_TRY(gemm<T>(st, false, false, n, n, n, T(1), LS, n, nn, Rm, n, 0, T(0), nullptr, 0, 0, ER, n, nn, 2));
        hipLaunchKernelGGL((k_endpoint_final<T>), dim3(grid_for(nn)), dim3(256), 0, st, nn, ER, ER + nn, I1,
                           I1 + (long)M * nn);
        LAUNCH_CHECK();
    } else {
        NEGF_TRY(conv_strip_launch<T>(n, n_tau, tg->kind, tg->kind == NEGF_TAU_POWER ? tg->block : 1, d_tau, d_w,
                                      Sc, G_in, I1, st));
        NEGF_TRY(gemm<T>(st, false, false, n, n, n, T(1), St, n, 0, G_in, n, nn, T(1), I1, n, nn, I1, n, nn, n_tau));
    }

    // ---------------- G0 + Q[G0, I1] in the eigenbasis, rotate back, mix
    const T* Ct = nullptr;
    if (sizeof(T) == 8) {
        Ct = (const T*)C;
    } else {
        float* Cf;
        NEGF_TRY(scratch_t(ctx, "dy_Cf", nn, &Cf));
        NEGF_TRY(to_f32(C, Cf, nn, st));
        Ct = (const T*)Cf;
    }
    NEGF_TRY(gemm<T>(st, true, false, n, n, n, T(1), Ct, n, 0, I1, n, nn, T(0), nullptr, 0, 0, It, n, nn, n_tau));
    double *Ea, *Eb, *dec, *cpre;
    NEGF_TRY(scratch_t(ctx, "dy_Ea", (size_t)n * n_tau, &Ea));
    NEGF_TRY(scratch_t(ctx, "dy_Eb", (size_t)n * n_tau, &Eb));
    NEGF_TRY(scratch_t(ctx, "dy_dec", (size_t)n * n_tau, &dec));
    NEGF_TRY(scratch_t(ctx, "dy_cpre", (size_t)n, &cpre));
    hipLaunchKernelGGL(k_scan_tables, dim3(grid_for((long)n * n_tau)), dim3(256), 0, st, n, n_tau, d_tau, tg->beta,
                       eps, mu, Ea, Eb, dec, cpre);
    LAUNCH_CHECK();
    // G0 + Q[G0, I1] in the eigenbasis: In read once and Out written once where a
    // chunk of 32 fits in registers, else the chunked kernel that rereads In
    const unsigned sblk = (unsigned)((nn + 15) / 16);
    // n >= 16: the rows of the decay tables a workgroup needs (at most two) are
    // staged in LDS, 6 n_tau doubles
    const size_t tsm = n >= 16 ? sizeof(double) * 6 * (size_t)n_tau : 0;
    auto scan_reg = [&](auto kern) -> int {
        static bool attr = false;
        if (!attr) {
            HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024));
            attr = true;
        }
        hipLaunchKernelGGL(kern, dim3(sblk), dim3(512), tsm, st, n, n_tau, It, I1, d_w, d_hL, d_hR, Ea, Eb, dec, cpre,
                           eps, mu, C);
        return NEGF_OK;
    };
    if (n_tau <= 32 * 17 && n >= 16)
        NEGF_TRY(scan_reg(k_eig_scan_reg<T, 17, true>));
    else if (n_tau <= 32 * 17)
        NEGF_TRY(scan_reg(k_eig_scan_reg<T, 17, false>));
    else if (n_tau <= 32 * 33 && n >= 16)
        NEGF_TRY(scan_reg(k_eig_scan_reg<T, 33, true>));
    else if (n_tau <= 32 * 33)
        NEGF_TRY(scan_reg(k_eig_scan_reg<T, 33, false>));
    else
        hipLaunchKernelGGL((k_eig_scan_chunked<T>), dim3(sblk), dim3(256), 0, st, n, n_tau, It, I1, d_w, d_hL, d_hR,
                           Ea, Eb, dec, cpre, eps, mu, C);
    LAUNCH_CHECK();
    NEGF_TRY(gemm<T>(st, false, false, n, n, n, (T)alpha, Ct, n, 0, I1, n, nn, (T)(1.0 - alpha), G_in, n, nn, G_out,
                     n, nn, n_tau));
    if (symmetrize && n > 0) {
        const int nt = (n + 31) / 32, npair = nt * (nt + 1) / 2;
        const int chunk = (int)std::min<long>(n_tau, 0x7fffffffL / npair);
        for (int s0 = 0; s0 < n_tau; s0 += chunk) {
            const int ns = min(chunk, n_tau - s0);
            hipLaunchKernelGGL((k_symmetrize<T>), dim3((unsigned)((long)npair * ns)), dim3(256), 0, st, n, nt, npair,
                               G_out + (long)s0 * nn);
            LAUNCH_CHECK();
        }
    }
    return NEGF_OK;
}

// Galitskii-Migdal energy and particle number of G into out[0], out[1] (device);
// stream-ordered, no host synchronisation once the weights are on the device.
template <class T>
int energy_launch(negf_ctx* ctx, const negf_tau_grid_t* tg, int n, int sigma, const double* h, const double* V,
                  const T* G, const T* Sc, double* out, hipStream_t st) {
    const int n_tau = tg->n_tau;
    std::vector<double> w, hL, hR;
    grid_tables(tg, w, hL, hR);
    void* dw = nullptr;
    NEGF_TRY(upload_cached(ctx, "en_w", w.data(), sizeof(double) * n_tau, st, &dw));
    double* part;
    const int nI = (n + 31) / 32;
    // sized for n up to 1024 at once, so that systems of a batch share one buffer
    NEGF_TRY(scratch_t(ctx, "en_part", (size_t)2 * n_tau * std::max(nI, 32), &part));
    hipLaunchKernelGGL((k_energy_slices<T>), dim3((unsigned)((long)n_tau * nI)), dim3(256), 0, st, n, n_tau, nI, Sc, G,
                       part);
    LAUNCH_CHECK();
    double* rowpart;
    // sized for n up to 1024 at once, so that systems of a batch share one buffer
    NEGF_TRY(scratch_t(ctx, "en_rowpart", (size_t)5 * std::max(n, 1024), &rowpart));
    hipLaunchKernelGGL((k_energy_rows<T>), dim3(n), dim3(256), 0, st, n, sigma, h, V, G + (long)(n_tau - 1) * n * n,
                       rowpart);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, st, n, n_tau, sigma, (const double*)dw, part,
                       (const double*)rowpart, out);
    LAUNCH_CHECK();
    return NEGF_OK;
}

template <class T>
int energy_run(negf_ctx* ctx, const negf_tau_grid_t* tg, int n, int sigma, const double* h, const double* V,
               const T* G, const T* Sc, double* E, double* N, hipStream_t st) {
    double* out;
    NEGF_TRY(scratch_t(ctx, "en_out", 2, &out));
    NEGF_TRY(energy_launch<T>(ctx, tg, n, sigma, h, V, G, Sc, out, st));
    double hres[2];
    HIP_TRY(hipMemcpyAsync(hres, out, sizeof(hres), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *E = hres[0];
    *N = hres[1];
    return NEGF_OK;
}

template <class T>
int density_run(int n, int n_tau, int sigma, const double* W, const T* G, double* out, hipStream_t st) {
    hipLaunchKernelGGL((k_density<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, sigma, W,
                       G + (long)(n_tau - 1) * n * n, out);
    LAUNCH_CHECK();
    return NEGF_OK;
}
template int density_run<double>(int, int, int, const double*, const double*, double*, hipStream_t);
template int density_run<float>(int, int, int, const double*, const float*, double*, hipStream_t);

template int dyson_run<double>(negf_ctx*, const negf_tau_grid_t*, int, int, const double*, const double*,
                               const double*, const double*, double, const double*, const double*, const double*,
                               double, int, int, double*, hipStream_t);
template int dyson_run<float>(negf_ctx*, const negf_tau_grid_t*, int, int, const double*, const double*,
                              const double*, const double*, double, const double*, const float*, const float*,
                              double, int, int, float*, hipStream_t);
template int energy_launch<double>(negf_ctx*, const negf_tau_grid_t*, int, int, const double*, const double*,
                                   const double*, const double*, double*, hipStream_t);
template int energy_launch<float>(negf_ctx*, const negf_tau_grid_t*, int, int, const double*, const double*,
                                  const float*, const float*, double*, hipStream_t);
template int energy_run<double>(negf_ctx*, const negf_tau_grid_t*, int, int, const double*, const double*,
                                const double*, const double*, double*, double*, hipStream_t);
template int energy_run<float>(negf_ctx*, const negf_tau_grid_t*, int, int, const double*, const double*,
                               const float*, const float*, double*, double*, hipStream_t);

}  // namespace negf
