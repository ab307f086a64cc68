// cmh_mdn.hpp -- constants, parameter layout and launchers of the
// mixture-density network used by the learned birth proposal.
#pragma once

#include <algorithm>

#include "cmh_common.hpp"

namespace cmh {

constexpr int kMdnWin = 64;             // envelope samples per station
constexpr int kMdnIn = 9 * kMdnWin;     // 3x3 stations x 64 = 576 features
constexpr int kMdnHid = 256;            // hidden width
constexpr int kMdnK = 8;                // mixture components
constexpr int kMdnOutPad = 64;          // 8 x 7 outputs padded to 64
constexpr int kMdnBg = 3;               // background events per training pair
constexpr int kMdnTScale = 32;          // window step and time unit, samples
constexpr int kMdnSplitRows = 256;      // batch rows per split of a gradient reduction, at least
constexpr int kMdnMaxSplits = 32;       // splits at most
constexpr int kMdnWgradSlots = 512;     // weight-gradient workgroups per product, at most
constexpr long kMdnBigTiles = 1024;     // 128 x 128 GEMM tiles from this many workgroups on
// clamps of the log standard deviations (x, y in units of ds; t in units of
// 32 samples): sigma_xy in [0.025, 1.5] ds, sigma_t in [0.5, 32] samples
constexpr float kMdnSloXY = -3.6888794541139363f;
constexpr float kMdnShiXY = 0.4054651081081644f;
constexpr float kMdnSloT = -4.1588830833596715f;
constexpr float kMdnShiT = 0.0f;
// the same sd clamps as plain ratios for the binary64 mixture table, and the
// table's clamps of the means: x, y within kMdnMuXY spacings of the anchor's
// station, t in [tau + 32 kMdnMuTLo, tau + 32 kMdnMuTHi]
constexpr double kMdnSdLoXY = 0.025, kMdnSdHiXY = 1.5;
constexpr double kMdnSdLoT = 0.5 / 32.0, kMdnSdHiT = 1.0;
constexpr double kMdnMuXY = 2.0, kMdnMuTLo = -1.0, kMdnMuTHi = 3.0;

// FP32 parameter blob: for layer l, W[l] (fout x fin, row-major, the
// layer's output index first) then b[l]; np floats.  The blob is followed by
// the Adam first and second moments (np floats each).  BF16 copies of the
// four weight matrices live in a separate array (offsets Wh[l], nh values).
struct MdnLayout {
    long W[4], b[4], Wh[4];
    long WhT[4];      // BF16 copies of layers 1..3 transposed, [fin][fout] (-1: none)
    int fin[4], fout[4];
    long np, nh;
};
MdnLayout mdn_layout();
// The whole network for M rows of features in one fused kernel (inference):
// head output O [M][64] fp32 only.
hipError_t mdn_infer(const float *params, const __bf16 *hcopy, const __bf16 *X, int M, float *O,
                     hipStream_t s);

struct MdnBuffers {
    float *Z[3];      // pre-activations, M x 256
    __bf16 *A[3];     // GELU activations, M x 256
    float *O;         // head output, M x 64
    __bf16 *dO;       // d loss / d head output, M x 64
    __bf16 *dH[2];    // M x 256
    float *loss;      // M
    float *part;      // split partial sums of every gradient: mdn_part_floats(M)
};
int mdn_splits(int M, int Mo, int N, int *per);
size_t mdn_part_floats(int M);

hipError_t mdn_init(float *params, __bf16 *hcopy, uint32_t seed, hipStream_t s);
hipError_t mdn_refresh_copies(const float *params, __bf16 *hcopy, hipStream_t s);
hipError_t mdn_forward(const float *params, const __bf16 *hcopy, const __bf16 *X, int M,
                       const MdnBuffers &B, hipStream_t s);
hipError_t mdn_backward(const float *params, const __bf16 *hcopy, const __bf16 *X, const float *Zt,
                        int M, const MdnBuffers &B, float *grad, hipStream_t s);
hipError_t mdn_adam(float *params, __bf16 *hcopy, const float *grad, int step, float lr,
                    hipStream_t s);
hipError_t mdn_pairs(const Geo &g, uint32_t seed, long first, int count, __bf16 *X, float *Zt,
                     hipStream_t s);
hipError_t anchor_features(const Geo &g, const void *trace, int f64, int ntau, long first, int count,
                           __bf16 *X, double *w, hipStream_t s);
hipError_t mixture_table(const Geo &g, int ntau, long first, int rows, const float *O, double *T,
                         hipStream_t s);

}  // namespace cmh
