// 6D Poisson-disk PST (Sec. 4 "PST pre-sampling": the template is a 6D
// Poisson-disk sample of the unit ball), by dart throwing.
//
// Candidates are rows 1, 2, ... of the i.i.d. template stream (pst_sample's
// Philox rows, uniform in the unit ball); the origin is accepted first; a
// candidate is accepted iff its squared distance to every point accepted
// before it is >= r_min^2.  Distances are taken on the sampler's lattice
// (p = a 2^-24, a odd integers below 2^24): differences stay below 2^25, so
// every square and the six-term sum (< 6 * 2^50) are exact in binary64 and
// the decision is exact.
//
// One workgroup walks the stream in batches of 512 candidates.  Per batch:
// every lane tests its candidate against all points accepted so far (staged
// through LDS in chunks, every lane reading the same row), and against the
// earlier candidates of its own batch (a 512 x 512 conflict bit matrix in
// LDS); one lane then settles the batch in stream order (a candidate is
// accepted iff it is far from everything accepted before and conflicts with
// no earlier candidate accepted in this batch), and the accepted candidates
// are appended in order.
#include "common.h"

namespace rose {

constexpr int kPoissonBatch = 512;
constexpr int kPoissonStage = 1024;  // accepted rows staged in LDS at a time
constexpr double kLattice = 16777216.0;  // 2^24

__global__ __launch_bounds__(kPoissonBatch) void k_pst_poisson(const float* cand, int32_t max_cand, int32_t n,
                                                               double d2, float* out, int32_t* result) {
    __shared__ float cb[kPoissonBatch * 6];
    __shared__ float stage[kPoissonStage * 6];
    __shared__ uint64_t conf[kPoissonBatch][kPoissonBatch / 64];
    __shared__ uint64_t farm[kPoissonBatch / 64];
    __shared__ uint64_t accm[kPoissonBatch / 64];
    __shared__ int count_s, count_prev_s, drawn_s, done_s;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // rows written by this workgroup are read back through L1-bypassing loads
    const volatile float* out_v = out;
    for (int64_t e = t; e < 6 * (int64_t)n; e += kPoissonBatch) out[e] = 0.0f;
    if (t == 0) {
        count_s = 1;  // the origin
        drawn_s = 0;
        done_s = (n <= 1 || max_cand < 1) ? 1 : 0;
    }
    __syncthreads();
    for (int base = 1; base <= max_cand; base += kPoissonBatch) {
        if (done_s) break;
        const int c = base + t;
        const bool valid = c <= max_cand;
        double a[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const float v = valid ? cand[6 * (int64_t)c + d] : 0.0f;
            cb[6 * t + d] = v;
            a[d] = (double)v * kLattice;
        }
        // far from every accepted point?
        bool far = valid;
        const int cnt = count_s;
        for (int k0 = 0; k0 < cnt; k0 += kPoissonStage) {
            const int kn = min(kPoissonStage, cnt - k0);
            __syncthreads();
            for (int e = t; e < 6 * kn; e += kPoissonBatch) stage[e] = out_v[6 * (int64_t)k0 + e];
            __syncthreads();
            for (int k = 0; k < kn; ++k) {
                double sq = 0.0;
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const double df = a[d] - (double)stage[6 * k + d] * kLattice;
                    sq = fma(df, df, sq);
                }
                far = far && (sq >= d2);
            }
        }
        __syncthreads();
        // conflicts with the earlier candidates of this batch
        for (int w = 0; w < kPoissonBatch / 64; ++w) {
            uint64_t bits = 0;
            for (int b = 0; b < 64; ++b) {
                const int i = w * 64 + b;
                if (i >= t) break;
                double sq = 0.0;
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const double df = a[d] - (double)cb[6 * i + d] * kLattice;
                    sq = fma(df, df, sq);
                }
                if (sq < d2) bits |= 1ull << b;
            }
            conf[t][w] = bits;
        }
        const uint64_t fb = __ballot(far);
        if (lane == 0) farm[wave] = fb;
        __syncthreads();
        if (t == 0) {
            uint64_t acc[kPoissonBatch / 64] = {0, 0, 0, 0, 0, 0, 0, 0};
            int cnt2 = count_s, last = -1;
            for (int j = 0; j < kPoissonBatch && base + j <= max_cand; ++j) {
                last = j;
                if ((farm[j >> 6] >> (j & 63)) & 1ull) {
                    bool ok = true;
                    for (int w = 0; w <= (j >> 6) && ok; ++w) ok = (conf[j][w] & acc[w]) == 0;
                    if (ok) {
                        acc[j >> 6] |= 1ull << (j & 63);
                        if (++cnt2 == n) break;
                    }
                }
            }
            for (int w = 0; w < kPoissonBatch / 64; ++w) accm[w] = acc[w];
            count_prev_s = count_s;
            count_s = cnt2;
            drawn_s = base + last;
            if (cnt2 == n || base + kPoissonBatch > max_cand) done_s = 1;
        }
        __syncthreads();
        if ((accm[wave] >> lane) & 1ull) {
            int pos = count_prev_s;
            for (int w = 0; w < wave; ++w) pos += __popcll(accm[w]);
            pos += __popcll(accm[wave] & ((1ull << lane) - 1ull));
#pragma unroll
            for (int d = 0; d < 6; ++d) out[6 * (int64_t)pos + d] = cb[6 * t + d];
        }
        __syncthreads();
    }
    if (t == 0) {
        result[0] = count_s;
        result[1] = drawn_s;
    }
}

}  // namespace rose

using namespace rose;

extern "C" {

rose_status pst_poisson(int32_t n, uint64_t seed, double r_min, int32_t max_candidates, float* work_dev,
                        float* out_dev, int32_t* result_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(work_dev && out_dev && result_dev, ROSE_E_ARG, "pst_poisson: NULL argument");
    ROSE_REQUIRE(n >= 1 && n <= ROSE_MAX_PARTICLES, ROSE_E_ARG, "pst_poisson: n = %d out of [1, %d]", n,
                 ROSE_MAX_PARTICLES);
    ROSE_REQUIRE(max_candidates >= 0 && max_candidates <= (1 << 24), ROSE_E_ARG,
                 "pst_poisson: max_candidates = %d out of [0, 2^24]", max_candidates);
    ROSE_REQUIRE(r_min >= 0.0 && r_min <= 2.0, ROSE_E_ARG, "pst_poisson: r_min must be in [0, 2]");
    // the threshold on the lattice, as the definition states it
    const double d2 = ceil(r_min * r_min * 281474976710656.0);
    rose_status st = launch_pst_sample((int64_t)max_candidates + 1, seed, work_dev, s);
    if (st != ROSE_OK) return st;
    hipLaunchKernelGGL(k_pst_poisson, dim3(1), dim3(kPoissonBatch), 0, s, work_dev, max_candidates, n, d2, out_dev,
                       result_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

}  // extern "C"
