// cmh_mdn.hip -- the learned birth proposal's network: a mixture-density
// MLP (576 -> 256 -> 256 -> 256 -> 8 Gaussian components over (x, y, t)),
// its training pairs and its input features.
//
//   k_gemm          C = op(A) op(B), BF16 operands on 16x16x32 MFMA tiles with
//                   FP32 accumulation, fused bias / GELU / GELU-backward epilogues,
//                   the bias gradient's column sums in the weight-gradient product
//   k_mdn_loss      mixture negative log-likelihood and its gradient
//   k_sum_jobs      the fixed-order sums of every gradient's split partials
//   k_adam_all      Adam on FP32 master weights, BF16 copies refreshed
//   k_sim_pairs     simulator-generated (window features, event) pairs
//   k_anchor_feat   window features and weights of an instance's anchors
//   k_mdn_init      Glorot-uniform initial weights from Philox
//
// Feature definition (both for pairs and anchors): for the 3x3 block of
// stations around a centre station (row-major), the log envelope
// e[n] = ln(sigma^2 + mean(s[n..n+3]^2)) - ln(sigma^2) over 64 samples from
// the window start, rounded to binary32 and then to BF16.
#include "cmh_common.hpp"
#include "cmh_mdn.hpp"

#include <math.h>

namespace cmh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline double gelu_d(double z) { return 0.5 * z * (1.0 + erf(z * M_SQRT1_2)); }
__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * (float)M_SQRT1_2)); }
__device__ inline float gelu_grad_f(float z)
{
    return 0.5f * (1.0f + erff(z * (float)M_SQRT1_2)) +
           z * expf(-0.5f * z * z) * (float)(0.5 * M_2_SQRTPI * M_SQRT1_2);
}

// -------------------------------------------------------------------- GEMM
// C[M][N] = sum_k op(A)[m][k] op(B)[k][n].  op(A)[m][k] = TA ? A[k*lda + m]
// : A[m*lda + k]; op(B)[k][n] = TB ? B[n*ldb + k] : B[k*ldb + n].  A
// workgroup of four waves (2 x 2) computes a (2 WM) x (2 WN) tile, each wave
// WM x WN as (WM/16) x (WN/16) MFMA 16x16x32 BF16 tiles with FP32
// accumulators.  k-steps of KS (whole MFMA k-slices of 32, taken in
// ascending order) go through double-buffered LDS: the next step's global
// loads are in flight while the current step's MFMAs run, one barrier per
// step; longer steps keep more loads in flight per barrier.  Loads are 16 bytes per lane along the operand's
// contiguous dimension, so the contiguous extents (M for TA, K otherwise,
// and N for !TB) and the leading dimensions must be multiples of 8.
// EPI 0: C (fp32).  EPI 1: Z = C + bias (fp32) and GELU(Z) as BF16 into Cb.
// EPI 2: C + bias (fp32).  EPI 3: the backward through GELU, BF16 C * GELU'(Z)
// into Cb, Z (fp32, row pitch ldc) passed as `bias`; C is not written.
// Split K: workgroup z sums k in [z kper, (z + 1) kper) and writes its
// partial product to C + z M ldc (EPI 0 only).  With TA, EPI 0 and colsum
// given (64-row tiles), the first column of workgroups also sums A over its
// k range for each of its M rows into colsum[z M + i] (the bias gradient of
// a weight-gradient product): thread t adds a quarter of row t / 4 of each
// step's tile in order, then the four quarters by a butterfly.
template <bool TA, bool TB, int EPI, int WM, int WN, int KS = 32>
__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, const __bf16 *__restrict__ A, int lda, const __bf16 *__restrict__ B,
       int ldb, float *__restrict__ C, int ldc, const float *__restrict__ bias,
       __bf16 *__restrict__ Cb, int ldcb, int kper, float *__restrict__ colsum)
{
    static_assert(KS % 32 == 0, "k-steps of whole MFMA k-slices");
    constexpr int TMR = 2 * WM, TNC = 2 * WN;       // workgroup tile
    constexpr int NVA = TMR * KS / 2048;            // 16-byte loads per thread per step (A)
    constexpr int NVB = TNC * KS / 2048;            //                                  (B)
    constexpr int FA = WM / 16, FB = WN / 16;       // MFMA tiles per wave
    constexpr int P = KS + 8;                       // LDS row pitch (bank spread)
    __shared__ __attribute__((aligned(16))) __bf16 sA[2][TMR][P];
    __shared__ __attribute__((aligned(16))) __bf16 sB[2][TNC][P];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i0 = blockIdx.y * TMR, j0 = blockIdx.x * TNC;
    const int wi = (wave >> 1) * WM, wj = (wave & 1) * WN;
    f32x4 acc[FA][FB];
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const __bf16 zero = (__bf16)0.0f;
    const int kbeg = blockIdx.z * kper;
    const int kend = min(K, kbeg + kper);
    C += (long)blockIdx.z * M * ldc;
    constexpr bool CS = TA && EPI == 0 && TMR * 4 == 256;  // one thread per row quarter
    const bool do_cs = CS && colsum != nullptr && blockIdx.x == 0;
    float cs = 0.f;

    // An operand stored k-strided (A for TA, B for !TB) is loaded as blocks of
    // 4 k-rows x 8 contiguous entries per thread (when the step holds exactly
    // one such block per thread per four vectors) and transposed in registers,
    // so that LDS takes 8-byte rows of 4 k's instead of 2-byte scalars.
    constexpr bool BLKA = TA && NVA % 4 == 0, BLKB = !TB && NVB % 4 == 0;
    bf16x8 ra[NVA], rb[NVB];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < NVA; ++u) {
            const int v = tid + 256 * u;
            ra[u] = (bf16x8){zero, zero, zero, zero, zero, zero, zero, zero};
            if (BLKA) {  // block u / 4 of this thread, k-row u % 4
                const int blk = tid + 256 * (u / 4);
                const int k4 = 4 * (blk / (TMR / 8)), m8 = 8 * (blk % (TMR / 8));
                const int gk = k0 + k4 + u % 4, gi = i0 + m8;
                if (gk < kend && gi < M) ra[u] = *(const bf16x8 *)&A[(long)gk * lda + gi];
            } else if (TA) {  // A[k][m]: 8 m's at one k
                const int kq = v / (TMR / 8), m8 = 8 * (v % (TMR / 8));
                const int gk = k0 + kq, gi = i0 + m8;
                if (gk < kend && gi < M) ra[u] = *(const bf16x8 *)&A[(long)gk * lda + gi];
            } else {   // A[m][k]: 8 k's of one row
                const int r = v / (KS / 8), k8 = 8 * (v % (KS / 8));
                const int gi = i0 + r, gk = k0 + k8;
                if (gi < M && gk < kend) ra[u] = *(const bf16x8 *)&A[(long)gi * lda + gk];
            }
        }
#pragma unroll
        for (int u = 0; u < NVB; ++u) {
            const int v = tid + 256 * u;
            rb[u] = (bf16x8){zero, zero, zero, zero, zero, zero, zero, zero};
            if (TB) {  // B[n][k]: 8 k's of one row
                const int r = v / (KS / 8), k8 = 8 * (v % (KS / 8));
                const int gj = j0 + r, gk = k0 + k8;
                if (gj < N && gk < kend) rb[u] = *(const bf16x8 *)&B[(long)gj * ldb + gk];
            } else if (BLKB) {
                const int blk = tid + 256 * (u / 4);
                const int k4 = 4 * (blk / (TNC / 8)), n8 = 8 * (blk % (TNC / 8));
                const int gk = k0 + k4 + u % 4, gj = j0 + n8;
                if (gk < kend && gj < N) rb[u] = *(const bf16x8 *)&B[(long)gk * ldb + gj];
            } else {   // B[k][n]: 8 n's at one k
                const int kq = v / (TNC / 8), n8 = 8 * (v % (TNC / 8));
                const int gk = k0 + kq, gj = j0 + n8;
                if (gk < kend && gj < N) rb[u] = *(const bf16x8 *)&B[(long)gk * ldb + gj];
            }
        }
    };
    // rows q of a 4 x 8 block (r[0..3]: k-rows) as 4 k-values each, into
    // dst[q][0..3] (8-byte stores)
    auto store_blk = [&](const bf16x8 *r, __bf16 (*dst)[P], int k4) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bf16x4 col = (bf16x4){r[0][q], r[1][q], r[2][q], r[3][q]};
            *(bf16x4 *)&dst[q][k4] = col;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NVA; ++u) {
            const int v = tid + 256 * u;
            if (BLKA) {
                if (u % 4 == 0) {
                    const int blk = tid + 256 * (u / 4);
                    const int k4 = 4 * (blk / (TMR / 8)), m8 = 8 * (blk % (TMR / 8));
                    store_blk(&ra[u], &sA[buf][m8], k4);
                }
            } else if (TA) {
                const int kq = v / (TMR / 8), m8 = 8 * (v % (TMR / 8));
#pragma unroll
                for (int q = 0; q < 8; ++q) sA[buf][m8 + q][kq] = ra[u][q];
            } else {
                *(bf16x8 *)&sA[buf][v / (KS / 8)][8 * (v % (KS / 8))] = ra[u];
            }
        }
#pragma unroll
        for (int u = 0; u < NVB; ++u) {
            const int v = tid + 256 * u;
            if (TB) {
                *(bf16x8 *)&sB[buf][v / (KS / 8)][8 * (v % (KS / 8))] = rb[u];
            } else if (BLKB) {
                if (u % 4 == 0) {
                    const int blk = tid + 256 * (u / 4);
                    const int k4 = 4 * (blk / (TNC / 8)), n8 = 8 * (blk % (TNC / 8));
                    store_blk(&rb[u], &sB[buf][n8], k4);
                }
            } else {
                const int kq = v / (TNC / 8), n8 = 8 * (v % (TNC / 8));
#pragma unroll
                for (int q = 0; q < 8; ++q) sB[buf][n8 + q][kq] = rb[u][q];
            }
        }
    };

    int cur = 0;
    if (kbeg < kend) {
        load(kbeg);
        store(0);
    }
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += KS) {
        const bool more = k0 + KS < kend;
        if (more) load(k0 + KS);           // in flight during the MFMAs below
        // k-slices of 32 in ascending order: the accumulation order of one
        // slice per step
#pragma unroll
        for (int ks = 0; ks < KS / 32; ++ks) {
            if (k0 + 32 * ks >= kend) break;  // the same in every lane
            const int kk = 32 * ks + 8 * (lane >> 4);
            bf16x8 fa[FA], fb[FB];
#pragma unroll
            for (int a = 0; a < FA; ++a)
                fa[a] = *(const bf16x8 *)&sA[cur][wi + 16 * a + (lane & 15)][kk];
#pragma unroll
            for (int b = 0; b < FB; ++b)
                fb[b] = *(const bf16x8 *)&sB[cur][wj + 16 * b + (lane & 15)][kk];
#pragma unroll
            for (int a = 0; a < FA; ++a)
#pragma unroll
                for (int b = 0; b < FB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b],
                                                                         0, 0, 0);
        }
        if constexpr (CS) {
            if (do_cs) {  // the same in every thread of the workgroup
                const int r = tid >> 2, q4 = tid & 3;
#pragma unroll
                for (int c = 0; c < KS / 32; ++c) {
                    const bf16x8 v = *(const bf16x8 *)&sA[cur][r][q4 * (KS / 4) + 8 * c];
#pragma unroll
                    for (int e = 0; e < 8; ++e) cs += (float)v[e];
                }
            }
        }
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    if constexpr (CS) {
        if (do_cs) {
            cs += __shfl_xor(cs, 1, 64);
            cs += __shfl_xor(cs, 2, 64);
            const int r = tid >> 2;
            if ((tid & 3) == 0 && i0 + r < M) colsum[(long)blockIdx.z * M + i0 + r] = cs;
        }
    }
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wi + 16 * a + 4 * (lane >> 4) + v;
                const int j = j0 + wj + 16 * b + (lane & 15);
                if (i >= M || j >= N) continue;
                float z = acc[a][b][v];
                if (EPI == 3) {  // dH = C * GELU'(Z), Z read through `bias` with row pitch ldc
                    Cb[(long)i * ldcb + j] = (__bf16)(z * gelu_grad_f(bias[(long)i * ldc + j]));
                    continue;
                }
                if (EPI != 0) z += bias[j];
                C[(long)i * ldc + j] = z;
                if (EPI == 1) Cb[(long)i * ldcb + j] = (__bf16)gelu_f(z);
            }
}

// Several fixed-order split sums in one launch: element q of job j is
// out[j][q] = sum over z (ascending) of part[j][z n_j + q].
struct SumJobs {
    const float *part[8];
    float *out[8];
    long n[8], start[9];
    int nz[8];
    int njobs;
};

__global__ void k_sum_jobs(SumJobs J)
{
    const long total = J.start[J.njobs];
    for (long g = blockIdx.x * (long)blockDim.x + threadIdx.x; g < total;
         g += (long)gridDim.x * blockDim.x) {
        int j = 0;
        while (j + 1 < J.njobs && g >= J.start[j + 1]) ++j;
        const long q = g - J.start[j], n = J.n[j];
        const float *part = J.part[j];
        float acc = 0.f;
#pragma unroll 8
        for (int z = 0; z < J.nz[j]; ++z) acc += part[(long)z * n + q];
        J.out[j][q] = acc;
    }
}

// Mixture negative log-likelihood of the targets and its gradient w.r.t. the
// head outputs, per sample: eight lanes per sample, lane k taking component
// k, the sums and maxima over a sample's components by butterflies within
// its eight lanes.  Head layout, component k: [7k] logit, [7k+1..3] means,
// [7k+4..6] log standard deviations, clamped to [slo_d, shi_d].  Gradients
// are divided by M (mean loss).
__device__ inline float group8_max(float v)
{
    for (int off = 1; off < 8; off <<= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline float group8_sum(float v)
{
    for (int off = 1; off < 8; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(256)
k_mdn_loss(int M, const float *__restrict__ O, int ldo, const float *__restrict__ Zt,
           float *__restrict__ loss, __bf16 *__restrict__ dO, int lddo)
{
    static_assert(kMdnK == 8, "one lane per component, eight per sample");
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int m = (int)(t >> 3), k = (int)(t & 7);
    const bool live = m < M;
    const int mm = live ? m : M - 1;  // every lane takes part in the butterflies
    const float *o = O + (long)mm * ldo + 7 * k;
    float ov[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) ov[c] = o[c];
    const float z[3] = {Zt[3 * (long)mm], Zt[3 * (long)mm + 1], Zt[3 * (long)mm + 2]};
    const float slo[3] = {kMdnSloXY, kMdnSloXY, kMdnSloT}, shi[3] = {kMdnShiXY, kMdnShiXY, kMdnShiT};
    const float lmax = group8_max(ov[0]);
    const float lse = lmax + logf(group8_sum(expf(ov[0] - lmax)));
    float l = ov[0] - lse, u[3], is[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float sd = fminf(fmaxf(ov[4 + d], slo[d]), shi[d]);
        is[d] = expf(-sd);
        u[d] = (z[d] - ov[1 + d]) * is[d];
        l += -0.5f * u[d] * u[d] - sd - 0.9189385332046727f;
    }
    const float best = group8_max(l);
    const float logp = best + logf(group8_sum(expf(l - best)));
    if (!live) return;
    if (k == 0) loss[m] = -logp;
    const float inv = 1.0f / (float)M;
    __bf16 *g = dO + (long)m * lddo;
    const float gam = expf(l - logp);
    const float pik = expf(ov[0] - lse);
    g[7 * k] = (__bf16)((pik - gam) * inv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        g[7 * k + 1 + d] = (__bf16)(-gam * u[d] * is[d] * inv);
        const bool free = ov[4 + d] > slo[d] && ov[4 + d] < shi[d];
        g[7 * k + 4 + d] = (__bf16)(free ? -gam * (u[d] * u[d] - 1.0f) * inv : 0.0f);
    }
    for (int c = 7 * kMdnK + k; c < lddo; c += 8) g[c] = (__bf16)0.0f;
}

// Adam (Kingma & Ba) with bias correction on FP32 master weights.
// Adam over the whole FP32 parameter blob (every layer's weights and bias,
// moments mo and ve laid out alike) in one pass; a weight's BF16 copy is
// refreshed at its place in hcopy.
struct AdamCopies {
    long w[4], nw[4], wh[4];  // layer weights: blob offset, count, offset in hcopy
    long wt[4];               // offset of the transposed copy in hcopy (-1: none)
    int fin[4], fout[4];
};

__global__ void k_adam_all(long n, float *__restrict__ w, float *__restrict__ mo,
                           float *__restrict__ ve, const float *__restrict__ g,
                           __bf16 *__restrict__ hcopy, AdamCopies cp, float lr, float b1, float b2,
                           float eps, float c1, float c2)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x) {
        const float gq = g[q];
        const float m = b1 * mo[q] + (1.f - b1) * gq;
        const float v = b2 * ve[q] + (1.f - b2) * gq * gq;
        mo[q] = m;
        ve[q] = v;
        const float wn = w[q] - lr * (m / c1) / (sqrtf(v / c2) + eps);
        w[q] = wn;
#pragma unroll
        for (int l = 0; l < 4; ++l)
            if (q >= cp.w[l] && q < cp.w[l] + cp.nw[l]) {
                const long r = q - cp.w[l];  // output row r / fin, input r % fin
                hcopy[cp.wh[l] + r] = (__bf16)wn;
                if (cp.wt[l] >= 0)
                    hcopy[cp.wt[l] + (r % cp.fin[l]) * cp.fout[l] + r / cp.fin[l]] = (__bf16)wn;
            }
    }
}

__global__ void k_to_bf16(long n, const float *__restrict__ w, __bf16 *__restrict__ wb)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x)
        wb[q] = (__bf16)w[q];
}

// w[fout][fin] as BF16, transposed: wt[i][o] = w[o][i].
__global__ void k_to_bf16_t(long n, int fin, int fout, const float *__restrict__ w,
                            __bf16 *__restrict__ wt)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x)
        wt[(q % fin) * fout + q / fin] = (__bf16)w[q];
}

// Glorot-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)), from
// Philox under key (seed, 0x80000004), counter (parameter index, 0, 0, 0);
// biases zero; padded head rows zero.
__global__ void k_mdn_init(float *__restrict__ W, long n, int fan_in, int fan_out, int rows_live,
                           long offset, uint32_t seed)
{
    const double a = sqrt(6.0 / (double)(fan_in + fan_out));
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x) {
        if (q / fan_in >= rows_live) {
            W[q] = 0.f;
            continue;
        }
        uint32_t c[4] = {(uint32_t)(offset + q), (uint32_t)((offset + q) >> 32), 0u, 0u};
        philox10(c, seed, 0x80000004u);
        W[q] = (float)((2.0 * unit_open(c[0], c[1]) - 1.0) * a);
    }
}

// --------------------------------------------------------------- features
// Rounds a binary64 feature to binary32 and then to BF16.
__device__ inline __bf16 feat_bf16(double v) { return (__bf16)(float)v; }

// Edge class of a training pair from a uniform u: class 0 (all nine block
// stations) when 16u < 8, else 16u - 7 in the order (ex, ey) = (-1,-1)
// (0,-1) (1,-1) (-1,0) (1,0) (-1,1) (0,1) (1,1); ex = -1 drops the block's
// left column and puts the domain edge half a spacing left of the centre.
__device__ inline void edge_class(double u, int *ex, int *ey)
{
    int k = (int)floor(u * 16.0);
    k = k > 15 ? 15 : k;
    if (k < 8) {
        *ex = 0;
        *ey = 0;
        return;
    }
    k -= 8;
    const int tx[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
    const int ty[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
    *ex = tx[k];
    *ey = ty[k];
}

// One training pair per wave: a local world around a centre station at the
// origin (3x3 block of stations at spacing ds, minus the row / column beyond
// the domain edge of its edge class), one target event within one spacing
// of the centre and kMdnBg background events anywhere that reaches the
// block, the present stations' traces over samples [0, 67) of the window,
// and the 576 window features (0 for a missing station).  Draws: key (seed,
// 0x80000003); counter (pair, 0, 0, c) for the events (c = 0 target x, y;
// c = 1 target t, magnitude; c = 2 + b background event b x, y; c = 2 +
// kMdnBg + b its t, magnitude; c = 8 the edge class); counter (pair, 1 +
// station, n / 2, 0) for the noise.  Events, arrivals and envelope sums in
// binary64; the noise and the features in binary32 (they end as BF16).
__global__ void __launch_bounds__(64)
k_sim_pairs(Geo g, uint32_t seed, long first, __bf16 *__restrict__ X, float *__restrict__ Zt)
{
    __shared__ double s_ev[kMdnBg + 1][4];
    __shared__ double s_arr[kMdnBg + 1][9][3];
    __shared__ float s_q[9][kMdnWin + 4];
    const long p = first + blockIdx.x;
    const int lane = threadIdx.x;
    uint32_t cm[4] = {(uint32_t)p, (uint32_t)(p >> 32), 0u, 8u};
    philox10(cm, seed, 0x80000003u);
    int ex, ey;
    edge_class(unit_open(cm[0], cm[1]), &ex, &ey);
    if (lane <= kMdnBg) {
        uint32_t c0[4] = {(uint32_t)p, (uint32_t)(p >> 32), 0u, (uint32_t)(lane == 0 ? 0 : 2 + (lane - 1))};
        uint32_t c1[4] = {(uint32_t)p, (uint32_t)(p >> 32), 0u,
                          (uint32_t)(lane == 0 ? 1 : 2 + kMdnBg + (lane - 1))};
        philox10(c0, seed, 0x80000003u);
        philox10(c1, seed, 0x80000003u);
        const double ux = unit_open(c0[0], c0[1]), uy = unit_open(c0[2], c0[3]);
        const double ut = unit_open(c1[0], c1[1]), um = unit_open(c1[2], c1[3]);
        const double reach = lane == 0 ? g.ds : 1.5 * g.ds + g.rc;
        const double xlo = ex < 0 ? -0.5 * g.ds : -reach, xhi = ex > 0 ? 0.5 * g.ds : reach;
        const double ylo = ey < 0 ? -0.5 * g.ds : -reach, yhi = ey > 0 ? 0.5 * g.ds : reach;
        s_ev[lane][0] = xlo + ux * (xhi - xlo);
        s_ev[lane][1] = ylo + uy * (yhi - ylo);
        s_ev[lane][2] = lane == 0 ? -16.0 + ut * 80.0
                                  : -(double)(g.ts + 8) + ut * (double)(kMdnWin + g.ts + 16);
        s_ev[lane][3] = g.mmin - log(um) / g.mrate;
    }
    __syncthreads();
    // per (event, station): reach, arrival, first sample and amplitude, the
    // same for every sample of the station
    if (lane < 9 * (kMdnBg + 1)) {
        const int b = lane % 9, q = lane / 9;
        const int dx = b % 3 - 1, dy = b / 3 - 1;
        const double sx = (double)dx * g.ds, sy = (double)dy * g.ds;
        const double ddx = s_ev[q][0] - sx, ddy = s_ev[q][1] - sy;
        const double d = sqrt(ddx * ddx + ddy * ddy);
        const double a = s_ev[q][2] + d / g.vel;
        s_arr[q][b][0] = d < g.rc ? a : NAN;   // NaN: out of reach
        s_arr[q][b][1] = ceil(a);
        s_arr[q][b][2] = s_ev[q][3] * exp(-d / g.atten);
    }
    __syncthreads();
    // noise of samples 2h and 2h + 1 of a station from one Box-Muller pair;
    // from here on binary32 (the features are rounded to BF16), the envelope
    // sums E in binary64
    const int nsamp = kMdnWin + 3, npair = (nsamp + 1) / 2;
    for (int e = lane; e < 9 * npair; e += 64) {
        const int b = e / npair, hn = e % npair;
        const int dx = b % 3 - 1, dy = b / 3 - 1;
        if ((ex != 0 && dx == ex) || (ey != 0 && dy == ey)) continue;
        uint32_t c[4] = {(uint32_t)p, (uint32_t)(p >> 32), (uint32_t)(1 + b), (uint32_t)hn};
        philox10(c, seed, 0x80000003u);
        const double u1 = unit_open(c[0], c[1]), u2 = unit_open(c[2], c[3]);
        const float rad = sqrtf(-2.0f * logf((float)u1));
        float sn, cs;
        sincosf((float)(2.0 * M_PI * u2), &sn, &cs);
        for (int o = 0; o < 2; ++o) {
            const int n = 2 * hn + o;
            if (n >= nsamp) break;
            double E = 0.0;
            for (int q = 0; q <= kMdnBg; ++q) {
                const double a = s_arr[q][b][0];
                if (!(a == a)) continue;
                const double n0 = s_arr[q][b][1];
                if ((double)n < n0 || (double)n >= n0 + g.ts) continue;
                const double amp = s_arr[q][b][2];
                const double env = exp(-((double)n - a) / g.decay);
                E += (amp * env) * (amp * env);
            }
            const float zz = rad * (o ? sn : cs);
            const float sv = sqrtf((float)(g.sigma2 + E)) * zz;
            s_q[b][n] = sv * sv;
        }
    }
    __syncthreads();
    const float is2 = (float)(1.0 / g.sigma2);
    __bf16 *xo = X + (long)blockIdx.x * kMdnIn;
    for (int e = lane; e < kMdnIn; e += 64) {
        const int b = e / kMdnWin, n = e % kMdnWin;
        const int dx = b % 3 - 1, dy = b / 3 - 1;
        if ((ex != 0 && dx == ex) || (ey != 0 && dy == ey)) {
            xo[e] = (__bf16)0.0f;
            continue;
        }
        // log(sigma^2 + m4) - log(sigma^2) as log1p(m4 / sigma^2): no cancellation
        const float m4 = (s_q[b][n] + s_q[b][n + 1] + s_q[b][n + 2] + s_q[b][n + 3]) * 0.25f;
        xo[e] = (__bf16)log1pf(m4 * is2);
    }
    if (lane == 0) {
        Zt[3 * (long)blockIdx.x + 0] = (float)(s_ev[0][0] / g.ds);
        Zt[3 * (long)blockIdx.x + 1] = (float)(s_ev[0][1] / g.ds);
        Zt[3 * (long)blockIdx.x + 2] = (float)(s_ev[0][2] / (double)kMdnTScale);
    }
}

// Window features and weight of anchors first .. first + count - 1 of an
// instance: anchor a = (station c = a / ntau, any station in row-major
// order; window start tau = 32 (a mod ntau)).  Block stations off the grid
// give 0.  Weight: 1e-3 + mean over the 576 features of max(0, f - 1).
template <typename TraceT>
__global__ void __launch_bounds__(64)
k_anchor_feat(Geo g, const TraceT *__restrict__ trace, int ntau, long first,
              __bf16 *__restrict__ X, double *__restrict__ wout)
{
    __shared__ double s_f[kMdnIn];
    const long a = first + blockIdx.x;
    const int lane = threadIdx.x;
    const int c = (int)(a / ntau), ti = (int)(a % ntau);
    const int cx = c % g.nsx, cy = c / g.nsx;
    const long tau = (long)kMdnTScale * ti;
    const double ls2 = log(g.sigma2);
    // the lane's kMdnIn / 64 features: every raw trace element loaded first
    // (stations off the grid read the anchor's own first element, unused),
    // then the features in the same summation order
    constexpr int K = kMdnIn / 64;
    static_assert(K * 64 == kMdnIn, "features split evenly over the lanes");
    TraceT raw[K][4];
    bool on[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = lane + 64 * k;
        const int b = e / kMdnWin, n = e % kMdnWin;
        const int ix = cx + b % 3 - 1, iy = cy + b / 3 - 1;
        on[k] = ix >= 0 && ix < g.nsx && iy >= 0 && iy < g.nsy;
        const TraceT *row = trace + (on[k] ? ((long)iy * g.nsx + ix) * g.N + tau + n
                                           : ((long)cy * g.nsx + cx) * g.N + tau);
#pragma unroll
        for (int u = 0; u < 4; ++u) raw[k][u] = row[u];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = lane + 64 * k;
        double f = 0.0;
        if (on[k]) {
            double acc = 0.0;
            for (int u = 0; u < 4; ++u) {
                const double v = (double)raw[k][u];
                acc += v * v;
            }
            f = log(g.sigma2 + acc * 0.25) - ls2;
        }
        const __bf16 fb = feat_bf16(f);
        X[(long)blockIdx.x * kMdnIn + e] = fb;
        s_f[e] = (double)(float)fb;
    }
    __syncthreads();
    double s = 0.0;
    for (int e = lane; e < kMdnIn; e += 64) s += s_f[e] > 1.0 ? s_f[e] - 1.0 : 0.0;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) wout[blockIdx.x] = 1e-3 + s / (double)kMdnIn;
}

// Mixture table rows of anchors first .. first + rows - 1 from the head
// outputs O[rows][64]: per component k, (mean x, y, t, sd x, y, t, log
// weight, cumulative weight) in absolute units.  Means are clamped to the
// anchor's station +- kMdnMuXY spacings and to [tau + 32 kMdnMuTLo, tau + 32
// kMdnMuTHi]; log sds to their training clamps.
__global__ void k_mixture_table(Geo g, int ntau, long first, int rows, const float *__restrict__ O,
                                double *__restrict__ T)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const long a = first + r;
    const int c = (int)(a / ntau);
    const double sx = station_pos(c % g.nsx, g.ds), sy = station_pos(c / g.nsx, g.ds);
    const double tau = (double)kMdnTScale * (double)(a % ntau);
    const float *o = O + (long)r * kMdnOutPad;
    double lmax = -1e300;
    for (int k = 0; k < kMdnK; ++k) lmax = fmax(lmax, (double)o[7 * k]);
    double se = 0.0;
    for (int k = 0; k < kMdnK; ++k) se += exp((double)o[7 * k] - lmax);
    const double lse = lmax + log(se);
    const double slo[3] = {log(kMdnSdLoXY), log(kMdnSdLoXY), log(kMdnSdLoT)};
    const double shi[3] = {log(kMdnSdHiXY), log(kMdnSdHiXY), log(kMdnSdHiT)};
    double *out = T + (long)r * kMdnK * 8;
    double cum = 0.0;
    for (int k = 0; k < kMdnK; ++k) {
        const double mx = fmin(fmax((double)o[7 * k + 1], -kMdnMuXY), kMdnMuXY);
        const double my = fmin(fmax((double)o[7 * k + 2], -kMdnMuXY), kMdnMuXY);
        const double mt = fmin(fmax((double)o[7 * k + 3], kMdnMuTLo), kMdnMuTHi);
        out[8 * k + 0] = sx + g.ds * mx;
        out[8 * k + 1] = sy + g.ds * my;
        out[8 * k + 2] = tau + (double)kMdnTScale * mt;
        for (int d = 0; d < 3; ++d) {
            const double ls = fmin(fmax((double)o[7 * k + 4 + d], slo[d]), shi[d]);
            out[8 * k + 3 + d] = (d < 2 ? g.ds : (double)kMdnTScale) * exp(ls);
        }
        const double lp = (double)o[7 * k] - lse;
        cum = cum + exp(lp);
        out[8 * k + 6] = lp;
        out[8 * k + 7] = cum;
    }
}

// ------------------------------------------------------------- launchers
// Tile choice: 128 x 128 workgroup tiles once they still give at least
// kMdnBigTiles workgroups (large row counts: inference over anchors), else
// (the training batch) 32 x 64 with k-steps of 64, twice the workgroups of
// 64 x 64 tiles and five resident per CU, or 64 x 64 with steps of 128 where
// an operand is stored k-strided, so that the grid fills the device.
template <bool TA, bool TB, int EPI>
static hipError_t gemm(int M, int N, int K, const __bf16 *A, int lda, const __bf16 *B, int ldb,
                       float *C, int ldc, const float *bias, __bf16 *Cb, int ldcb, hipStream_t s)
{
    const long big = (long)((M + 127) / 128) * ((N + 127) / 128);
    if (N >= 128 && big >= kMdnBigTiles) {
        const dim3 grid((N + 127) / 128, (M + 127) / 128, 1);
        k_gemm<TA, TB, EPI, 64, 64, 32><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc,
                                                              bias, Cb, ldcb, K, nullptr);
    } else if (TA || !TB) {  // a k-strided operand: 64 x 64 tiles, whose steps of 128 hold
                             // whole 4 x 8 blocks per thread for the register transposes
        const dim3 grid((N + 63) / 64, (M + 63) / 64, 1);
        k_gemm<TA, TB, EPI, 32, 32, 128><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc,
                                                               bias, Cb, ldcb, K, nullptr);
    } else {
        const dim3 grid((N + 63) / 64, (M + 31) / 32, 1);
        k_gemm<TA, TB, EPI, 16, 32, 64><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc,
                                                              bias, Cb, ldcb, K, nullptr);
    }
    return hipGetLastError();
}

static unsigned grid_for(long n) { return (unsigned)std::min<long>((n + 255) / 256, 8192); }

// Row splits of a weight-gradient product C[Mo][N] over a batch of M rows:
// as many as keep the product's 64 x 64 tiles times the splits within
// kMdnWgradSlots workgroups (one round of two per CU), at most
// kMdnMaxSplits, with chunks of at least kMdnSplitRows rows (a multiple of
// 32).  The same for every call with the same shape.
int mdn_splits(int M, int Mo, int N, int *per)
{
    const int tiles = ((Mo + 63) / 64) * ((N + 63) / 64);
    int z = std::max(1, kMdnWgradSlots / tiles);
    z = std::min(z, kMdnMaxSplits);
    z = std::min(z, (M + kMdnSplitRows - 1) / kMdnSplitRows);
    z = std::max(z, 1);
    int p = (M + z - 1) / z;
    p = (p + 31) / 32 * 32;
    *per = p;
    return (M + p - 1) / p;
}

// Weight gradient C[Mo][N] = sum over the batch of op(A)^T B and bias
// gradient db[Mo] = column sums of A[Mb][Mo], split over the batch into
// partial products (part) and partial sums (bpart) whose fixed-order sums
// are left to the job list J (summed by one launch for every gradient of a
// backward pass).
static hipError_t weight_grad(int Mo, int N, int Mb, const __bf16 *A, int lda, const __bf16 *B,
                              int ldb, float *C, float *db, float *part, float *bpart,
                              SumJobs &J, hipStream_t s)
{
    int per = 0;
    const int nz = mdn_splits(Mb, Mo, N, &per);
    const dim3 grid((N + 63) / 64, (Mo + 63) / 64, nz);
    k_gemm<true, false, 0, 32, 32, 128><<<grid, 256, 0, s>>>(Mo, N, Mb, A, lda, B, ldb,
                                                        nz > 1 ? part : C, N, nullptr, nullptr, 0,
                                                        per, nz > 1 ? bpart : db);
    hipError_t e = hipGetLastError();
    if (e || nz == 1) return e;
    int j = J.njobs++;
    J.part[j] = part; J.out[j] = C; J.n[j] = (long)Mo * N; J.nz[j] = nz;
    J.start[j + 1] = J.start[j] + J.n[j];
    j = J.njobs++;
    J.part[j] = bpart; J.out[j] = db; J.n[j] = Mo; J.nz[j] = nz;
    J.start[j + 1] = J.start[j] + J.n[j];
    return hipSuccess;
}

// Partial-sum floats one backward pass over M rows needs: every layer's
// weight- and bias-gradient splits side by side.
size_t mdn_part_floats(int M)
{
    const int fin[4] = {kMdnIn, kMdnHid, kMdnHid, kMdnHid};
    const int fout[4] = {kMdnHid, kMdnHid, kMdnHid, kMdnOutPad};
    size_t n = 0;
    for (int l = 0; l < 4; ++l) {
        int per = 0;
        const size_t nz = (size_t)mdn_splits(M, fout[l], fin[l], &per);
        n += nz * fin[l] * fout[l] + nz * fout[l];
    }
    return n;
}

MdnLayout mdn_layout()
{
    MdnLayout L;
    long o = 0;
    const int fin[4] = {kMdnIn, kMdnHid, kMdnHid, kMdnHid};
    const int fout[4] = {kMdnHid, kMdnHid, kMdnHid, kMdnOutPad};
    for (int l = 0; l < 4; ++l) {
        L.W[l] = o; L.fin[l] = fin[l]; L.fout[l] = fout[l];
        o += (long)fin[l] * fout[l];
        L.b[l] = o;
        o += fout[l];
    }
    L.np = o;
    long h = 0;
    for (int l = 0; l < 4; ++l) {
        L.Wh[l] = h;
        h += (long)L.fin[l] * L.fout[l];
    }
    // transposed copies for the backward pass's dA = dOut W products, after
    // the copies the inference kernel reads
    L.WhT[0] = -1;
    for (int l = 1; l < 4; ++l) {
        L.WhT[l] = h;
        h += (long)L.fin[l] * L.fout[l];
    }
    L.nh = h;
    return L;
}

hipError_t mdn_init(float *params, __bf16 *hcopy, uint32_t seed, hipStream_t s)
{
    const MdnLayout L = mdn_layout();
    hipError_t e = hipSuccess;
    for (int l = 0; l < 4 && !e; ++l) {
        const long n = (long)L.fin[l] * L.fout[l];
        const int live = l == 3 ? 7 * kMdnK : L.fout[l];
        k_mdn_init<<<grid_for(n), 256, 0, s>>>(params + L.W[l], n, L.fin[l],
                                              l == 3 ? 7 * kMdnK : L.fout[l], live, L.W[l], seed);
        e = hipGetLastError();
        if (!e) e = hipMemsetAsync(params + L.b[l], 0, sizeof(float) * L.fout[l], s);
    }
    // Adam moments
    if (!e) e = hipMemsetAsync(params + L.np, 0, sizeof(float) * 2 * L.np, s);
    if (!e) e = mdn_refresh_copies(params, hcopy, s);
    return e;
}

hipError_t mdn_refresh_copies(const float *params, __bf16 *hcopy, hipStream_t s)
{
    const MdnLayout L = mdn_layout();
    for (int l = 0; l < 4; ++l) {
        const long n = (long)L.fin[l] * L.fout[l];
        k_to_bf16<<<grid_for(n), 256, 0, s>>>(n, params + L.W[l], hcopy + L.Wh[l]);
        hipError_t e = hipGetLastError();
        if (e) return e;
        if (L.WhT[l] < 0) continue;
        k_to_bf16_t<<<grid_for(n), 256, 0, s>>>(n, L.fin[l], L.fout[l], params + L.W[l],
                                                hcopy + L.WhT[l]);
        if ((e = hipGetLastError())) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------- fused inference
// The whole network for a tile of kInfRows rows in one workgroup: layer 1
// streams the features and every layer streams its BF16 weights through
// double-buffered LDS chunks of 32 inputs, the hidden activations stay in
// LDS between layers (GELU(Z + b) rounded to BF16, as the layer-by-layer
// forward stores them), and only the head output (Z + b, fp32) goes to HBM.
// Eight waves as 4 x 2: a wave owns 32 rows x 128 outputs of a hidden layer
// (16 MFMA 16x16x32 tiles) and 32 rows x 32 outputs of the head; two waves
// per SIMD hide each other's LDS and barrier latency.
constexpr int kInfRows = 128;
// Offsets of layer l's BF16 weights and FP32 bias in the parameter blobs (the
// layout mdn_layout describes), as constants so that no layout object lives
// in the kernel's private memory.
__host__ __device__ constexpr long mdn_fin(int l) { return l == 0 ? kMdnIn : kMdnHid; }
__host__ __device__ constexpr long mdn_fout(int l) { return l == 3 ? kMdnOutPad : kMdnHid; }
__host__ __device__ constexpr long mdn_wh_off(int l)
{
    return (l > 0 ? (long)kMdnIn * kMdnHid : 0) + (l > 1 ? (long)(l - 1) * kMdnHid * kMdnHid : 0);
}
// the FP32 blob holds each layer's weights followed by its bias; the BF16 copy
// holds the weights alone
__host__ __device__ constexpr long mdn_b_off(int l)
{
    return mdn_wh_off(l) + (long)l * kMdnHid + mdn_fin(l) * mdn_fout(l);
}
constexpr int kInfPitch = kMdnHid + 8;  // LDS row pitch of the activations (bank spread)

__global__ void __launch_bounds__(512)
k_mdn_infer(int M, const __bf16 *__restrict__ X, const __bf16 *__restrict__ W,
            const float *__restrict__ params, float *__restrict__ out)
{
    extern __shared__ __attribute__((aligned(16))) __bf16 s_inf[];
    __bf16 (*sH)[kInfPitch] = (__bf16 (*)[kInfPitch])s_inf;                       // 128 x 264
    __bf16 (*sA)[kInfRows][40] = (__bf16 (*)[kInfRows][40])(s_inf + kInfRows * kInfPitch);
    __bf16 (*sB)[kMdnHid][40] = (__bf16 (*)[kMdnHid][40])(s_inf + kInfRows * kInfPitch +
                                                          2 * kInfRows * 40);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.x * kInfRows;
    const int wr = (wave >> 1) * 32;
    const __bf16 zero = (__bf16)0.0f;
    const bf16x8 z8 = (bf16x8){zero, zero, zero, zero, zero, zero, zero, zero};
    const int kk = 8 * (lane >> 4);

#pragma unroll
    for (int l = 0; l < 4; ++l) {  // unrolled: every layer's shape is a constant
        const int K = l == 0 ? kMdnIn : kMdnHid;
        const int NO = l == 3 ? kMdnOutPad : kMdnHid;
        const int wc = (wave & 1) * (NO / 2);
        const __bf16 *Wl = W + mdn_wh_off(l);  // [NO][K]
        constexpr int FA = 2;
        const int FB = NO / 32;          // 8 hidden, 2 head
        f32x4 acc[FA][8];
#pragma unroll
        for (int a = 0; a < FA; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
        // chunk loads: W rows (NO x 32), and for layer 1 the feature rows
        bf16x8 rb[2], ra;
        auto load = [&](int k0) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int v = tid + 512 * u, n = v >> 2;
                rb[u] = n < NO ? *(const bf16x8 *)&Wl[(long)n * K + k0 + 8 * (v & 3)] : z8;
            }
            if (l == 0) {
                const int r = tid >> 2, gr = r0 + r;
                ra = gr < M ? *(const bf16x8 *)&X[(long)gr * kMdnIn + k0 + 8 * (tid & 3)] : z8;
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int v = tid + 512 * u, n = v >> 2;
                if (n < NO) *(bf16x8 *)&sB[buf][n][8 * (v & 3)] = rb[u];
            }
            if (l == 0) *(bf16x8 *)&sA[buf][tid >> 2][8 * (tid & 3)] = ra;
        };
        int cur = 0;
        load(0);
        store(0);
        __syncthreads();
        for (int k0 = 0; k0 < K; k0 += 32) {
            const bool more = k0 + 32 < K;
            if (more) load(k0 + 32);
            bf16x8 fa[FA];
#pragma unroll
            for (int a = 0; a < FA; ++a) {
                const int row = wr + 16 * a + (lane & 15);
                fa[a] = l == 0 ? *(const bf16x8 *)&sA[cur][row][kk]
                               : *(const bf16x8 *)&sH[row][k0 + kk];
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                if (b < FB) {  // one weight fragment live at a time
                    const bf16x8 fb = *(const bf16x8 *)&sB[cur][wc + 16 * b + (lane & 15)][kk];
#pragma unroll
                    for (int a = 0; a < FA; ++a)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb, acc[a][b],
                                                                           0, 0, 0);
                }
            }
            if (more) store(cur ^ 1);
            __syncthreads();  // also: every read of sH by this layer is done
            cur ^= 1;
        }
        const float *bias = params + mdn_b_off(l);
        if (l < 3) {  // GELU(Z + b) as BF16 into the activations
#pragma unroll
            for (int a = 0; a < FA; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = wr + 16 * a + 4 * (lane >> 4) + v;
                        const int j = wc + 16 * b + (lane & 15);
                        sH[i][j] = (__bf16)gelu_f(acc[a][b][v] + bias[j]);
                    }
            __syncthreads();
        } else {
#pragma unroll
            for (int a = 0; a < FA; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = r0 + wr + 16 * a + 4 * (lane >> 4) + v;
                        const int j = wc + 16 * b + (lane & 15);
                        if (i < M) out[(long)i * kMdnOutPad + j] = acc[a][b][v] + bias[j];
                    }
        }
    }
}

size_t mdn_infer_lds()
{
    return sizeof(__bf16) * ((size_t)kInfRows * kInfPitch + 2 * kInfRows * 40 + 2 * kMdnHid * 40);
}

hipError_t mdn_infer(const float *params, const __bf16 *hcopy, const __bf16 *X, int M, float *O,
                     hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    const MdnLayout L = mdn_layout();
    for (int l = 0; l < 4; ++l)
        if (L.Wh[l] != mdn_wh_off(l) || L.b[l] != mdn_b_off(l)) return hipErrorInvalidValue;
    const size_t lds = mdn_infer_lds();
    hipError_t e = hipFuncSetAttribute((const void *)k_mdn_infer,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_mdn_infer<<<(M + kInfRows - 1) / kInfRows, 512, lds, s>>>(M, X, hcopy, params, O);
    return hipGetLastError();
}

// Forward pass for M rows of features.  Buffers: Z[l] fp32 pre-activations
// and A[l] BF16 activations of the three hidden layers, O fp32 head output.
hipError_t mdn_forward(const float *params, const __bf16 *hcopy, const __bf16 *X, int M,
                       const MdnBuffers &B, hipStream_t s)
{
    const MdnLayout L = mdn_layout();
    hipError_t e;
    const __bf16 *in = X;
    int kin = kMdnIn;
    for (int l = 0; l < 3; ++l) {
        e = gemm<false, true, 1>(M, kMdnHid, kin, in, kin, hcopy + L.Wh[l], kin, B.Z[l], kMdnHid,
                                 params + L.b[l], B.A[l], kMdnHid, s);
        if (e) return e;
        in = B.A[l];
        kin = kMdnHid;
    }
    return gemm<false, true, 2>(M, kMdnOutPad, kMdnHid, in, kMdnHid, hcopy + L.Wh[3], kMdnHid,
                                B.O, kMdnOutPad, params + L.b[3], nullptr, 0, s);
}

// Loss and gradients of the mean mixture NLL w.r.t. every parameter (into
// grad, laid out like the FP32 parameters).
hipError_t mdn_backward(const float *params, const __bf16 *hcopy, const __bf16 *X, const float *Zt,
                        int M, const MdnBuffers &B, float *grad, hipStream_t s)
{
    const MdnLayout L = mdn_layout();
    hipError_t e = mdn_forward(params, hcopy, X, M, B, s);
    if (e) return e;
    k_mdn_loss<<<(unsigned)(((long)M * 8 + 255) / 256), 256, 0, s>>>(M, B.O, kMdnOutPad, Zt, B.loss,
                                                                    B.dO, kMdnOutPad);
    if ((e = hipGetLastError())) return e;
    // Every gradient's partials get a region of B.part of their own, so that
    // one launch at the end sums them all (each in a fixed order).
    SumJobs J{};
    int per = 0;
    long nz = mdn_splits(M, kMdnOutPad, kMdnHid, &per);
    float *part = B.part;
    // head: dW4 = dO^T A3, db4 = sum dO, dA3 = dO W4
    e = weight_grad(kMdnOutPad, kMdnHid, M, B.dO, kMdnOutPad, B.A[2], kMdnHid, grad + L.W[3],
                    grad + L.b[3], part, part + nz * kMdnOutPad * kMdnHid, J, s);
    if (e) return e;
    part += nz * kMdnOutPad * kMdnHid + nz * kMdnOutPad;
    const __bf16 *dnext = B.dO;
    int nout = kMdnOutPad;
    for (int l = 2; l >= 0; --l) {
        // dA_l = dOut W_{l+1} (W_{l+1}'s transposed copy as the k-contiguous
        // operand); dH_l = dA_l * GELU'(Z_l)
        e = gemm<false, true, 3>(M, kMdnHid, nout, dnext, nout, hcopy + L.WhT[l + 1], nout,
                                 nullptr, kMdnHid, B.Z[l], B.dH[l & 1], kMdnHid, s);
        if (e) return e;
        const __bf16 *in = l == 0 ? X : B.A[l - 1];
        const int kin = l == 0 ? kMdnIn : kMdnHid;
        nz = mdn_splits(M, kMdnHid, kin, &per);
        e = weight_grad(kMdnHid, kin, M, B.dH[l & 1], kMdnHid, in, kin, grad + L.W[l],
                        grad + L.b[l], part, part + nz * kMdnHid * kin, J, s);
        if (e) return e;
        part += nz * kMdnHid * kin + nz * kMdnHid;
        dnext = B.dH[l & 1];
        nout = kMdnHid;
    }
    if (J.njobs == 0) return hipSuccess;
    k_sum_jobs<<<grid_for(J.start[J.njobs]), 256, 0, s>>>(J);
    return hipGetLastError();
}

hipError_t mdn_adam(float *params, __bf16 *hcopy, const float *grad, int step, float lr,
                    hipStream_t s)
{
    const MdnLayout L = mdn_layout();
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    AdamCopies cp;
    for (int l = 0; l < 4; ++l) {
        cp.w[l] = L.W[l];
        cp.nw[l] = (long)L.fin[l] * L.fout[l];
        cp.wh[l] = L.Wh[l];
        cp.wt[l] = L.WhT[l];
        cp.fin[l] = L.fin[l];
        cp.fout[l] = L.fout[l];
    }
    k_adam_all<<<grid_for(L.np), 256, 0, s>>>(L.np, params, params + L.np, params + 2 * L.np, grad,
                                              hcopy, cp, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mdn_pairs(const Geo &g, uint32_t seed, long first, int count, __bf16 *X, float *Zt,
                     hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    k_sim_pairs<<<count, 64, 0, s>>>(g, seed, first, X, Zt);
    return hipGetLastError();
}

hipError_t anchor_features(const Geo &g, const void *trace, int f64, int ntau, long first, int count,
                           __bf16 *X, double *w, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (f64)
        k_anchor_feat<double><<<count, 64, 0, s>>>(g, (const double *)trace, ntau, first, X, w);
    else
        k_anchor_feat<float><<<count, 64, 0, s>>>(g, (const float *)trace, ntau, first, X, w);
    return hipGetLastError();
}

hipError_t mixture_table(const Geo &g, int ntau, long first, int rows, const float *O, double *T,
                         hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    k_mixture_table<<<(rows + 127) / 128, 128, 0, s>>>(g, ntau, first, rows, O, T);
    return hipGetLastError();
}

}  // namespace cmh
