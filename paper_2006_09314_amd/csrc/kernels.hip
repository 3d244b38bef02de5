// Device kernels of the fracctl library, written for gfx950 (CDNA4):
// 64-wide wavefronts, FP64 matrix cores (v_mfma_f64_16x16x4f64), 160 KiB LDS.
#include "kernels.h"

#include <cstdint>
#include <mutex>
#include <utility>
#include <vector>

namespace fc {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Wavefront sum of a double through DPP moves (row shifts and row
// broadcasts, both 32-bit halves), the total read from lane 63 and returned
// to every lane.  Lanes whose DPP source is absent or masked add zero.
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline double dpp_take(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double wave_sum(double v) {
    v += dpp_take<0xb1>(v);          // quad_perm [1,0,3,2]
    v += dpp_take<0x4e>(v);          // quad_perm [2,3,0,1]: every lane holds its quad sum
    v += dpp_take<0x114>(v);         // row_shr:4
    v += dpp_take<0x118>(v);         // row_shr:8: lane 15 of a row holds the row sum
    v += dpp_take<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_take<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3: lane 63 holds the total
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}
typedef float flt4 __attribute__((ext_vector_type(4)));
// accumulator row of register v in lane l for v_mfma_f32_16x16x4f32
#define F32_ROW(l, v) (4 * ((l) >> 4) + (v))

// ---------------------------------------------------------------------------
// Batched FP64 GEMM on the matrix cores.
//
// A workgroup of WM x WN wavefronts owns a (32 WM) x (32 WN) tile of C; each
// wavefront owns a 32 x 32 sub-tile held as 2 x 2 MFMA 16x16 accumulators.
// K is consumed in chunks of 32 staged through LDS (coalesced global reads in
// the operand's storage order), the next chunk fetched into registers while
// the current one is used.  MFMA 16x16x4 f64 operand layout: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register v of
// lane l holds C[l / 16 + 4 v][l % 16] (checked by the layout self-test).
template <bool TA, bool TB, int WM, int WN>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int tile, int b, int kz, int kchunk,
                                          bool split) {
    constexpr int BM = 32 * WM, BN = 32 * WN, BK = 32, NT = 64 * WM * WN;
    constexpr int PA = BM * BK / NT, PB = BK * BN / NT;   // staged values per thread
    __shared__ double As[BK][BM + 1];
    __shared__ double Bs[BK][BN + 1];
    const int tilesM = (g.M + BM - 1) / BM;
    const int tm = tile % tilesM, tn = tile / tilesM;
    const long bo = b / g.inner, bi = b % g.inner;
    const double* __restrict__ A = g.A + bo * g.strideA + bi * g.strideAin;
    const double* __restrict__ B = g.B + bo * g.strideB + bi * g.strideBin;
    const double* __restrict__ d = g.d ? g.d + bo * g.strideD : nullptr;
    double* __restrict__ C = g.C + bo * g.strideC + bi * g.strideCin;
    long ldc = g.ldc;
    double alpha = g.alpha, beta = g.beta;
    const int kbeg = kz * kchunk, kend = min(g.K, kbeg + kchunk);
    if (split) {
        // partial product of this K slice -> part[kz][b] (M x N, ld M)
        C = g.part + ((long)kz * g.batch + b) * (long)g.M * g.N;
        ldc = g.M;
        alpha = 1.0;
        beta = 0.0;
    }
    const int row0 = tm * BM, col0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    dbl4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    // chunks of BK staged in LDS along the index contiguous in memory; the
    // next chunk is fetched into registers while the current one is used
    double pa[PA], pb[PB];
    auto a_ik = [&](int e, int& i, int& k) {
        if (!TA) { i = e % BM; k = e / BM; } else { k = e % BK; i = e / BK; }
    };
    auto b_kj = [&](int e, int& k, int& j) {
        if (!TB) { k = e % BK; j = e / BK; } else { j = e % BN; k = e / BN; }
    };
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            int i, k;
            a_ik(tid + u * NT, i, k);
            const int gi = row0 + i, gk = k0 + k;
            double v = 0.0;
            if (gi < g.M && gk < kend) {
                v = TA ? A[gk + (long)gi * g.lda] : A[gi + (long)gk * g.lda];
                if (d) v *= d[gk];
            }
            pa[u] = v;
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            int k, j;
            b_kj(tid + u * NT, k, j);
            const int gj = col0 + j, gk = k0 + k;
            pb[u] = (gj < g.N && gk < kend) ? (TB ? B[gj + (long)gk * g.ldb] : B[gk + (long)gj * g.ldb]) : 0.0;
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            int i, k;
            a_ik(tid + u * NT, i, k);
            As[k][i] = pa[u];
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            int k, j;
            b_kj(tid + u * NT, k, j);
            Bs[k][j] = pb[u];
        }
        __syncthreads();
        if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            // a reduction that ends inside the chunk stops at its last step
            // of four (the rest of the chunk holds zeros)
            if (k0 + 4 * kk >= kend) break;
            const int k = kk * 4 + (lane >> 4);
            const double a0 = As[k][wm * 32 + (lane & 15)];
            const double a1 = As[k][wm * 32 + 16 + (lane & 15)];
            const double b0 = Bs[k][wn * 32 + (lane & 15)];
            const double b1 = Bs[k][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    for (int mi = 0; mi < 2; ++mi)
        for (int ni = 0; ni < 2; ++ni)
            for (int v = 0; v < 4; ++v) {
                const int i = row0 + wm * 32 + mi * 16 + (lane >> 4) + 4 * v;
                const int j = col0 + wn * 32 + ni * 16 + (lane & 15);
                if (i < g.M && j < g.N) {
                    double r = alpha * acc[mi][ni][v];
                    if (beta != 0.0) r += beta * C[i + (long)j * ldc];
                    C[i + (long)j * ldc] = r;
                }
            }
}

template <bool TA, bool TB, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void gemm_kernel(GemmArgs g, int kchunk) {
    gemm_tile<TA, TB, WM, WN>(g, blockIdx.x, blockIdx.y, blockIdx.z, kchunk, gridDim.z > 1);
}

// Up to three independent plain products in one launch: grid.y picks the
// product, grid.x runs over the largest product's tiles times its batch
// (blocks beyond a product's own return at once).  Whole K per block; a
// product may be a strided (two-level) batch.
template <bool TA, bool TB, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void gemm_multi_kernel(GramJobs jobs) {
    const GemmArgs& g = jobs.g[blockIdx.y];
    const int tiles = ((g.M + 32 * WM - 1) / (32 * WM)) * ((g.N + 32 * WN - 1) / (32 * WN));
    if ((long)blockIdx.x >= (long)tiles * g.batch) return;
    gemm_tile<TA, TB, WM, WN>(g, blockIdx.x % tiles, blockIdx.x / tiles, 0, g.K, false);
}

hipError_t gemm_multi(bool transA, bool transB, const GramJobs& jobs, hipStream_t s) {
    long most = 0;
    for (int t = 0; t < jobs.count; ++t) {
        const GemmArgs& g = jobs.g[t];
        if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch < 1 || g.inner < 1 || g.d || g.lowp)
            return hipErrorInvalidValue;
        most = std::max(most, (long)((g.M + 31) / 32) * ((g.N + 31) / 32) * g.batch);
    }
    if (jobs.count <= 0) return hipSuccess;
    if (most > 0x7fffffffL) return hipErrorInvalidValue;
    const dim3 grid(most, jobs.count), block(64);
    if (!transA && !transB)
        hipLaunchKernelGGL((gemm_multi_kernel<false, false, 1, 1>), grid, block, 0, s, jobs);
    else if (!transA && transB)
        hipLaunchKernelGGL((gemm_multi_kernel<false, true, 1, 1>), grid, block, 0, s, jobs);
    else if (transA && !transB)
        hipLaunchKernelGGL((gemm_multi_kernel<true, false, 1, 1>), grid, block, 0, s, jobs);
    else
        hipLaunchKernelGGL((gemm_multi_kernel<true, true, 1, 1>), grid, block, 0, s, jobs);
    return hipGetLastError();
}

template <bool TA, bool TB, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void gemm32_kernel(GemmArgs g, int kchunk) {
    constexpr int BM = 32 * WM, BN = 32 * WN, BK = 16, NT = 64 * WM * WN;
    __shared__ float As[BK][BM + 1];
    __shared__ float Bs[BK][BN + 1];
    const int tilesM = (g.M + BM - 1) / BM;
    const int tm = blockIdx.x % tilesM, tn = blockIdx.x / tilesM;
    const int b = blockIdx.y;
    const long bo = b / g.inner, bi = b % g.inner;
    const double* __restrict__ A = g.A + bo * g.strideA + bi * g.strideAin;
    const double* __restrict__ B = g.B + bo * g.strideB + bi * g.strideBin;
    const double* __restrict__ d = g.d ? g.d + bo * g.strideD : nullptr;
    double* __restrict__ C = g.C + bo * g.strideC + bi * g.strideCin;
    long ldc = g.ldc;
    double alpha = g.alpha, beta = g.beta;
    const int kz = blockIdx.z;
    const int kbeg = kz * kchunk, kend = min(g.K, kbeg + kchunk);
    if (gridDim.z > 1) {
        // partial product of this K slice -> part[kz][b] (M x N, ld M)
        C = g.part + ((long)kz * g.batch + b) * (long)g.M * g.N;
        ldc = g.M;
        alpha = 1.0;
        beta = 0.0;
    }
    const int row0 = tm * BM, col0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    flt4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        for (int e = tid; e < BM * BK; e += NT) {
            int i, k;
            if (!TA) { i = e % BM; k = e / BM; } else { k = e % BK; i = e / BK; }
            const int gi = row0 + i, gk = k0 + k;
            double v = 0.0;
            if (gi < g.M && gk < kend) {
                v = TA ? A[gk + (long)gi * g.lda] : A[gi + (long)gk * g.lda];
                if (d) v *= d[gk];
            }
            As[k][i] = (float)v;
        }
        for (int e = tid; e < BK * BN; e += NT) {
            int j, k;
            if (!TB) { k = e % BK; j = e / BK; } else { j = e % BN; k = e / BN; }
            const int gj = col0 + j, gk = k0 + k;
            double v = 0.0;
            if (gj < g.N && gk < kend) v = TB ? B[gj + (long)gk * g.ldb] : B[gk + (long)gj * g.ldb];
            Bs[k][j] = (float)v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int k = kk * 4 + (lane >> 4);
            const float a0 = As[k][wm * 32 + (lane & 15)];
            const float a1 = As[k][wm * 32 + 16 + (lane & 15)];
            const float b0 = Bs[k][wn * 32 + (lane & 15)];
            const float b1 = Bs[k][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    for (int mi = 0; mi < 2; ++mi)
        for (int ni = 0; ni < 2; ++ni)
            for (int v = 0; v < 4; ++v) {
                const int i = row0 + wm * 32 + mi * 16 + F32_ROW(lane, v);
                const int j = col0 + wn * 32 + ni * 16 + (lane & 15);
                if (i < g.M && j < g.N) {
                    double r = alpha * (double)acc[mi][ni][v];
                    if (beta != 0.0) r += beta * C[i + (long)j * ldc];
                    C[i + (long)j * ldc] = r;
                }
            }
}

// sum of the split-K partial products: C = alpha sum_z part[z] + beta C
__global__ void splitk_reduce_kernel(GemmArgs g, int ksplit) {
    const long mn = (long)g.M * g.N;
    const long total = mn * g.batch;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const long b = e / mn, ij = e % mn;
        const int i = int(ij % g.M), j = int(ij / g.M);
        double s = 0.0;
        for (int z = 0; z < ksplit; ++z) s += g.part[((long)z * g.batch + b) * mn + ij];
        const long bo = b / g.inner, bi = b % g.inner;
        double* C = g.C + bo * g.strideC + bi * g.strideCin;
        double r = g.alpha * s;
        if (g.beta != 0.0) r += g.beta * C[i + (long)j * g.ldc];
        C[i + (long)j * g.ldc] = r;
    }
}

// 64 x 64 tiles (four wavefronts sharing their staged chunks) for large
// products, also where M or N is below 64 as long as such tiles pad no more
// than 32 x 32 ones (sizes in (32, 64] modulo 64): the batches of 54 x 54
// blocks of the Hadamard truncation's per-term Grams run on a quarter of
// the workgroups (measured: 64 solves at n = 1024 166 -> 169 solves/s)
template <bool TA, bool TB>
static hipError_t gemm_dispatch(const GemmArgs& g, hipStream_t s) {
    const long work = (long)g.M * g.N * g.batch;
    auto same_pad = [](int x) { return (x + 63) / 64 * 64 == (x + 31) / 32 * 32; };
    const bool big = work >= (1L << 20) &&
                     ((g.M >= 64 && g.N >= 64) || (same_pad(g.M) && same_pad(g.N)));
    const int BMN = big ? 64 : 32;
    const long tiles = (long)((g.M + BMN - 1) / BMN) * ((g.N + BMN - 1) / BMN);
    const long wgs = tiles * g.batch;
    int ksplit = 1;
    if (g.part && wgs < 256 && g.K >= 256) {
        ksplit = (int)std::min<long>(std::max<long>(1, 512 / wgs), g.K / 128);
        while (ksplit > 1 && (long)ksplit * g.batch * g.M * g.N > g.part_cap) --ksplit;
    }
    int kchunk = (g.K + ksplit - 1) / ksplit;
    kchunk = (kchunk + 15) / 16 * 16;
    ksplit = (g.K + kchunk - 1) / kchunk;
    if (g.lowp) {
        if (big)
            hipLaunchKernelGGL((gemm32_kernel<TA, TB, 2, 2>), dim3(tiles, g.batch, ksplit), dim3(256),
                               0, s, g, kchunk);
        else
            hipLaunchKernelGGL((gemm32_kernel<TA, TB, 1, 1>), dim3(tiles, g.batch, ksplit), dim3(64),
                               0, s, g, kchunk);
    } else if (big) {
        hipLaunchKernelGGL((gemm_kernel<TA, TB, 2, 2>), dim3(tiles, g.batch, ksplit), dim3(256), 0, s,
                           g, kchunk);
    } else {
        hipLaunchKernelGGL((gemm_kernel<TA, TB, 1, 1>), dim3(tiles, g.batch, ksplit), dim3(64), 0, s,
                           g, kchunk);
    }
    if (ksplit > 1) {
        const long total = (long)g.M * g.N * g.batch;
        const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, s, g, ksplit);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Products with a long reduction: C = alpha op(A) diag(d) op(B) + beta C
// with op(A) op(B) = A^T B (L = 0), A B^T (L = 1) or A B (L = 2),
// column-major operands, d (length K, optional) scaling the reduction index.
// One workgroup per 32 x 32 output tile.  K is taken in chunks of GR_KC:
// the workgroup stages the chunk's 32 rows of op(A) and 32 columns of
// op(B) (the latter already scaled by d) in LDS with coalesced loads, along
// whichever index is contiguous in memory, and fetches the next chunk into
// registers while its wavefronts run the current one on the FP64 matrix
// core (16x16x4; the wavefronts take the chunk's k-steps in turn, reading
// their operands from LDS in the matrix-core lane layout: lane l row/column
// l % 16, k = l / 16).  The wavefronts' partial tiles are summed in LDS in
// a fixed order (deterministic).  Batched over blockIdx.z with strides (d
// advances by strideD per batch entry).  The number of wavefronts per
// workgroup (8 or 16) is chosen by the autotuner per problem size.
constexpr int GR_KC = 128;          // K chunk staged in LDS
constexpr int GR_LD = GR_KC + 4;    // padded row of a staged chunk (doubles)

template <int L, int W>
__device__ __forceinline__ void gram_tile_staged(const GemmArgs& g, int tile, long b) {
    extern __shared__ double gram_sm[];   // As, Bs [32][GR_LD]; after the K loop: partial tiles
    constexpr int T = 64 * W;
    constexpr int PER = 32 * GR_KC / T;  // values per thread and operand per chunk
    constexpr bool a_kfast = (L == 0);   // op(A) row i is contiguous in k
    constexpr bool b_kfast = (L != 1);   // op(B) column j is contiguous in k
    double* As = gram_sm;
    double* Bs = gram_sm + 32 * GR_LD;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tilesM = (g.M + 31) / 32;
    const int i0 = (tile % tilesM) * 32, j0 = (tile / tilesM) * 32;
    const double* __restrict__ A = g.A + b * g.strideA;
    const double* __restrict__ B = g.B + b * g.strideB;
    const double* __restrict__ d = g.d ? g.d + b * g.strideD : nullptr;
    double* __restrict__ C = g.C + b * g.strideC;
    const int r16 = lane & 15, kq = lane >> 4;
    double pa[PER], pb[PER];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * T;
            {
                const int c = a_kfast ? e / GR_KC : e % 32, kk = kc + (a_kfast ? e % GR_KC : e / 32);
                const int i = i0 + c;
                pa[u] = (kk < g.K && i < g.M)
                            ? (a_kfast ? A[kk + (long)i * g.lda] : A[i + (long)kk * g.lda]) : 0.0;
            }
            {
                const int c = b_kfast ? e / GR_KC : e % 32, kk = kc + (b_kfast ? e % GR_KC : e / 32);
                const int j = j0 + c;
                double v = (kk < g.K && j < g.N)
                               ? (b_kfast ? B[kk + (long)j * g.ldb] : B[j + (long)kk * g.ldb]) : 0.0;
                if (d) v *= (kk < g.K) ? d[kk] : 0.0;
                pb[u] = v;
            }
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * T;
            As[(a_kfast ? e / GR_KC : e % 32) * GR_LD + (a_kfast ? e % GR_KC : e / 32)] = pa[u];
            Bs[(b_kfast ? e / GR_KC : e % 32) * GR_LD + (b_kfast ? e % GR_KC : e / 32)] = pb[u];
        }
    };
    dbl4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int kc = 0; kc < g.K; kc += GR_KC) {
        __syncthreads();   // the previous chunk has been read
        put();
        __syncthreads();
        if (kc + GR_KC < g.K) fetch(kc + GR_KC);
        for (int st = wave; st < GR_KC / 4; st += W) {
            const int k = 4 * st + kq;
            const double a0 = As[r16 * GR_LD + k], a1 = As[(16 + r16) * GR_LD + k];
            const double b0 = Bs[r16 * GR_LD + k], b1 = Bs[(16 + r16) * GR_LD + k];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    __syncthreads();   // the LDS now takes the partial tiles
    double* red = gram_sm;   // [W][4 blocks][4 regs][64 lanes]
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int v = 0; v < 4; ++v)
                red[((wave * 4 + 2 * x + y) * 4 + v) * 64 + lane] = acc[x][y][v];
    __syncthreads();
    // 32 x 32 outputs; accumulator v of lane l holds row (l >> 4) + 4 v,
    // column l & 15 of its 16 x 16 block
    for (int e = threadIdx.x; e < 2 * 2 * 4 * 64; e += T) {
        const int l = e & 63, v = (e >> 6) & 3, blk = e >> 8;
        const int x = blk >> 1, y = blk & 1;
        double sum = 0.0;
        for (int w = 0; w < W; ++w) sum += red[((w * 4 + blk) * 4 + v) * 64 + l];
        const int i = i0 + 16 * x + (l >> 4) + 4 * v, j = j0 + 16 * y + (l & 15);
        if (i < g.M && j < g.N) {
            double r = g.alpha * sum;
            if (g.beta != 0.0) r += g.beta * C[i + (long)j * g.ldc];
            C[i + (long)j * g.ldc] = r;
        }
    }
}

// The direct variant: no staging; its wavefronts split K in interleaved
// chunks of 16 and load their operands straight from memory into the
// matrix-core lane layout (lane l: row/column l % 16, k = l / 16), with no
// barrier in the K loop.  It keeps the edge where K is long and the tiles
// few (unfolding Grams of cores, K = r^2), where the staged variant spends
// a barrier pair per chunk.
constexpr int GR_DEPTH = 1;   // chunks loaded per wavefront before computing

template <int L, int GR_WAVES>
__device__ __forceinline__ void gram_tile_direct(const GemmArgs& g, int tile, long b) {
    extern __shared__ double gram_red[];   // [GR_WAVES][4 blocks][4 regs][64 lanes]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tilesM = (g.M + 31) / 32;
    const int i0 = (tile % tilesM) * 32, j0 = (tile / tilesM) * 32;
    const double* __restrict__ A = g.A + b * g.strideA;
    const double* __restrict__ B = g.B + b * g.strideB;
    const double* __restrict__ d = g.d ? g.d + b * g.strideD : nullptr;
    double* __restrict__ C = g.C + b * g.strideC;
    const int r16 = lane & 15, kq = lane >> 4;
    const int ia0 = i0 + r16, ia1 = i0 + 16 + r16;
    const int jb0 = j0 + r16, jb1 = j0 + 16 + r16;
    const bool va0 = ia0 < g.M, va1 = ia1 < g.M, vb0 = jb0 < g.N, vb1 = jb1 < g.N;
    // element (row i of op(A), k) is A[k + i lda] for L = 0, else A[i + k lda];
    // element (k, column j of op(B)) is B[j + k ldb] for L = 1, else B[k + j ldb]
    const long sa = (L == 0) ? 1 : g.lda, sb = (L == 1) ? g.ldb : 1;
    const double* a0p = A + (va0 ? ((L == 0) ? (long)ia0 * g.lda : ia0) : 0);
    const double* a1p = A + (va1 ? ((L == 0) ? (long)ia1 * g.lda : ia1) : 0);
    const double* b0p = B + (vb0 ? ((L == 1) ? jb0 : (long)jb0 * g.ldb) : 0);
    const double* b1p = B + (vb1 ? ((L == 1) ? jb1 : (long)jb1 * g.ldb) : 0);
    dbl4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int chunks = (g.K + 15) / 16;
    for (int base = wave; base < chunks; base += GR_WAVES * GR_DEPTH) {
        double a0[4 * GR_DEPTH], a1[4 * GR_DEPTH], b0[4 * GR_DEPTH], b1[4 * GR_DEPTH];
#pragma unroll
        for (int u = 0; u < 4 * GR_DEPTH; ++u) {
            const int k = 16 * (base + GR_WAVES * (u >> 2)) + 4 * (u & 3) + kq;
            const bool vk = k < g.K;
            a0[u] = (vk && va0) ? a0p[k * sa] : 0.0;
            a1[u] = (vk && va1) ? a1p[k * sa] : 0.0;
            b0[u] = (vk && vb0) ? b0p[k * sb] : 0.0;
            b1[u] = (vk && vb1) ? b1p[k * sb] : 0.0;
            if (d) {
                const double dk = vk ? d[k] : 0.0;
                b0[u] *= dk;
                b1[u] *= dk;
            }
        }
#pragma unroll
        for (int u = 0; u < 4 * GR_DEPTH; ++u) {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b0[u], acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b1[u], acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b0[u], acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], acc[1][1], 0, 0, 0);
        }
    }
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int v = 0; v < 4; ++v)
                gram_red[((wave * 4 + 2 * x + y) * 4 + v) * 64 + lane] = acc[x][y][v];
    __syncthreads();
    // 32 x 32 outputs, two per thread; accumulator v of lane l holds
    // row (l >> 4) + 4 v, column l & 15 of its 16 x 16 block
    for (int e = threadIdx.x; e < 2 * 2 * 4 * 64; e += 64 * GR_WAVES) {
        const int l = e & 63, v = (e >> 6) & 3, blk = e >> 8;
        const int x = blk >> 1, y = blk & 1;
        double sum = 0.0;
        for (int w = 0; w < GR_WAVES; ++w) sum += gram_red[((w * 4 + blk) * 4 + v) * 64 + l];
        const int i = i0 + 16 * x + (l >> 4) + 4 * v, j = j0 + 16 * y + (l & 15);
        if (i < g.M && j < g.N) {
            double r = g.alpha * sum;
            if (g.beta != 0.0) r += g.beta * C[i + (long)j * g.ldc];
            C[i + (long)j * g.ldc] = r;
        }
    }
}

template <int L, int W, bool S>
__device__ __forceinline__ void gram_tile(const GemmArgs& g, int tile, long b) {
    if constexpr (S) gram_tile_staged<L, W>(g, tile, b);
    else gram_tile_direct<L, W>(g, tile, b);
}

template <int L, int W, bool S>
__global__ __launch_bounds__(64 * W) void gram_kernel(GemmArgs g) {
    gram_tile<L, W, S>(g, blockIdx.x, blockIdx.z);
}

// Up to kMaxGramJobs independent products (each possibly a strided batch)
// in one launch: grid.y picks the product, grid.x runs over its tiles times
// its batch; blocks beyond a product's own count return at once.
template <int L, int W, bool S>
__global__ __launch_bounds__(64 * W) void gram_multi_kernel(GramJobs jobs) {
    const GemmArgs& g = jobs.g[blockIdx.y];
    const int tiles = ((g.M + 31) / 32) * ((g.N + 31) / 32);
    if ((long)blockIdx.x >= (long)tiles * g.batch) return;
    gram_tile<L, W, S>(g, (int)(blockIdx.x % tiles), (long)(blockIdx.x / tiles));
}

// Batches of diagonally scaled Grams C_q = alpha A^T diag(d_q) B + beta C_q
// that share A and B (strideA = strideB = 0; d_q at d + q strideD, C_q at
// C + q strideC): one workgroup per 32 x 32 output tile and group of QG
// consecutive terms.  The K chunks of A and B are staged in LDS once for
// the group (coalesced, the next chunk fetched into registers while the
// current one is used) with the group's QG chunks of d; every wavefront
// takes its k-steps for all QG terms, scaling its B operand by d_q in
// registers.  The group shares its operand loads and its barriers, so a
// batch runs on a quarter (QG = 4) or half of the workgroups, each doing
// QG times the matrix-core work: fewer compute units held for the batch,
// which leaves room for the kernels of concurrent solves.  Partial tiles
// are summed in LDS term by term in a fixed wavefront order (deterministic).
template <int W, int QG>
__device__ __forceinline__ void sgram_tile(const GemmArgs& g, int tile, int q0) {
    extern __shared__ double gram_sm[];   // As, Bs [32][GR_LD], Ds [QG][GR_KC]; then partial tiles
    constexpr int T = 64 * W;
    constexpr int PER = 32 * GR_KC / T;
    constexpr int PERD = (QG * GR_KC + T - 1) / T;
    double* As = gram_sm;
    double* Bs = gram_sm + 32 * GR_LD;
    double* Ds = gram_sm + 64 * GR_LD;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tilesM = (g.M + 31) / 32;
    const int i0 = (tile % tilesM) * 32, j0 = (tile / tilesM) * 32;
    const int nq = min(QG, g.batch - q0);
    const double* __restrict__ A = g.A;
    const double* __restrict__ B = g.B;
    const double* __restrict__ d = g.d + (long)q0 * g.strideD;
    const int r16 = lane & 15, kq = lane >> 4;
    double pa[PER], pb[PER], pd[PERD];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * T;
            const int c = e / GR_KC, kk = kc + e % GR_KC;
            const bool vk = kk < g.K;
            pa[u] = (vk && i0 + c < g.M) ? A[kk + (long)(i0 + c) * g.lda] : 0.0;
            pb[u] = (vk && j0 + c < g.N) ? B[kk + (long)(j0 + c) * g.ldb] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PERD; ++u) {
            const int e = threadIdx.x + u * T;
            const int t = e / GR_KC, kk = kc + e % GR_KC;
            pd[u] = (e < QG * GR_KC && t < nq && kk < g.K) ? d[kk + (long)t * g.strideD] : 0.0;
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * T;
            As[(e / GR_KC) * GR_LD + e % GR_KC] = pa[u];
            Bs[(e / GR_KC) * GR_LD + e % GR_KC] = pb[u];
        }
#pragma unroll
        for (int u = 0; u < PERD; ++u) {
            const int e = threadIdx.x + u * T;
            if (e < QG * GR_KC) Ds[e] = pd[u];
        }
    };
    dbl4 acc[QG][2][2];
#pragma unroll
    for (int t = 0; t < QG; ++t)
        for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y) acc[t][x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int kc = 0; kc < g.K; kc += GR_KC) {
        __syncthreads();   // the previous chunk has been read
        put();
        __syncthreads();
        if (kc + GR_KC < g.K) fetch(kc + GR_KC);
        for (int st = wave; st < GR_KC / 4; st += W) {
            const int k = 4 * st + kq;
            const double a0 = As[r16 * GR_LD + k], a1 = As[(16 + r16) * GR_LD + k];
            const double b0 = Bs[r16 * GR_LD + k], b1 = Bs[(16 + r16) * GR_LD + k];
#pragma unroll
            for (int t = 0; t < QG; ++t) {
                const double dk = Ds[t * GR_KC + k];
                const double c0 = b0 * dk, c1 = b1 * dk;
                acc[t][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, c0, acc[t][0][0], 0, 0, 0);
                acc[t][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, c1, acc[t][0][1], 0, 0, 0);
                acc[t][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, c0, acc[t][1][0], 0, 0, 0);
                acc[t][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, c1, acc[t][1][1], 0, 0, 0);
            }
        }
    }
    double* red = gram_sm;   // [W][4 blocks][4 regs][64 lanes], one term at a time
#pragma unroll
    for (int t = 0; t < QG; ++t) {
        __syncthreads();   // the LDS is free (staged chunks, or the previous term's partials)
        for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y)
                for (int v = 0; v < 4; ++v)
                    red[((wave * 4 + 2 * x + y) * 4 + v) * 64 + lane] = acc[t][x][y][v];
        __syncthreads();
        if (t < nq) {
            double* __restrict__ C = g.C + (long)(q0 + t) * g.strideC;
            for (int e = threadIdx.x; e < 2 * 2 * 4 * 64; e += T) {
                const int l = e & 63, v = (e >> 6) & 3, blk = e >> 8;
                const int x = blk >> 1, y = blk & 1;
                double sum = 0.0;
                for (int w = 0; w < W; ++w) sum += red[((w * 4 + blk) * 4 + v) * 64 + l];
                const int i = i0 + 16 * x + (l >> 4) + 4 * v, j = j0 + 16 * y + (l & 15);
                if (i < g.M && j < g.N) {
                    double r = g.alpha * sum;
                    if (g.beta != 0.0) r += g.beta * C[i + (long)j * g.ldc];
                    C[i + (long)j * g.ldc] = r;
                }
            }
        }
    }
}

// Up to kMaxGramJobs such batches in one launch: grid.y picks the batch,
// grid.x runs over its tiles times its term groups.
template <int W, int QG>
__global__ __launch_bounds__(64 * W) void sgram_multi_kernel(GramJobs jobs) {
    const GemmArgs& g = jobs.g[blockIdx.y];
    const int tiles = ((g.M + 31) / 32) * ((g.N + 31) / 32);
    const int groups = (g.batch + QG - 1) / QG;
    if ((long)blockIdx.x >= (long)tiles * groups) return;
    sgram_tile<W, QG>(g, (int)(blockIdx.x % tiles), (int)(blockIdx.x / tiles) * QG);
}

// ---------------------------------------------------------------------------
// Streaming products with a long reduction and a small right or output
// side: C = alpha op(A) op(B) + beta C with op(A) op(B) = A^T B (L = 0),
// A B^T (L = 1) or A B (L = 2), up to three jobs per launch.  This carries
// the mode transforms (A the n x n eigenvector matrix of a mode, stored as
// V or V^T so that A is read along its columns; B n x m) and the Gram-type
// products whose few output tiles would leave the GPU idle.  A workgroup of
// four wavefronts owns 32 rows of C and a chunk of KC values of K (every
// wavefront KC / 4 of them): each lane loads all of its A operands of the
// chunk (2 rows x STEPS steps of 4) before its first product, so the whole A
// panel is requested at once; the products run on the FP64 matrix core
// (16x16x4) for every 32-column block of C in turn (the upper 16 columns
// only where C has them), with the A operands in registers.  The four
// partial tiles are summed in LDS in a fixed order.  With K split over
// several chunks the partial tiles go to `part` and a second kernel adds
// them in chunk order, so the result does not depend on the schedule.  (A
// last-arriving workgroup could add them in the same launch, but the
// device-scope fence each workgroup then needs writes back its XCD's L2:
// measured, that costs more than the second launch.)
constexpr int TR_WAVES = 4;

template <int L, int STEPS>
__global__ __launch_bounds__(64 * TR_WAVES) void stream_kernel(StreamJobs jobs, int ksplit,
                                                               double* part, long pstride) {
    constexpr int KC = 4 * STEPS * TR_WAVES;
    __shared__ double red[TR_WAVES][4][4][64];
    const StreamJob& J = jobs.job[blockIdx.y];
    const int rblocks = (J.M + 31) / 32;
    const int rb = blockIdx.x / ksplit, kz = blockIdx.x % ksplit;
    if (rb >= rblocks) return;
    const int i0 = rb * 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int ia0 = i0 + r16, ia1 = i0 + 16 + r16;
    const bool va0 = ia0 < J.M, va1 = ia1 < J.M;
    const int m = J.N;
    const bool split = ksplit > 1;
    double* __restrict__ out = split ? part + ((long)blockIdx.y * ksplit + kz) * pstride : J.C;
    const long ldo = split ? J.M : J.ldc;
    // element (i, k) of op(A) and (k, j) of op(B)
    const long sa_i = (L == 0) ? J.lda : 1, sa_k = (L == 0) ? 1 : J.lda;
    const long sb_k = (L == 1) ? J.ldb : 1, sb_j = (L == 1) ? 1 : J.ldb;
    const int kend = min(J.K, (kz + 1) * KC);
    const int kw = kz * KC + 4 * STEPS * wave;   // this wavefront's first k
    double a0[STEPS], a1[STEPS];
#pragma unroll
    for (int u = 0; u < STEPS; ++u) {
        const int k = kw + 4 * u + kq;
        const bool vk = k < kend;
        a0[u] = (vk && va0) ? J.A[ia0 * sa_i + k * sa_k] : 0.0;
        a1[u] = (vk && va1) ? J.A[ia1 * sa_i + k * sa_k] : 0.0;
    }
    for (int c0 = 0; c0 < m; c0 += 32) {
        const int jb0 = c0 + r16, jb1 = c0 + 16 + r16;
        const bool vb0 = jb0 < m, vb1 = jb1 < m;
        const bool hi = c0 + 16 < m;   // the block's upper 16 columns exist
        dbl4 acc[2][2];
        for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
        double b0[STEPS], b1[STEPS];
#pragma unroll
        for (int u = 0; u < STEPS; ++u) {
            const int k = kw + 4 * u + kq;
            const bool vk = k < kend;
            b0[u] = (vk && vb0) ? J.B[k * sb_k + jb0 * sb_j] : 0.0;
            b1[u] = (hi && vk && vb1) ? J.B[k * sb_k + jb1 * sb_j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < STEPS; ++u) {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b0[u], acc[0][0], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b0[u], acc[1][0], 0, 0, 0);
        }
        if (hi) {
#pragma unroll
            for (int u = 0; u < STEPS; ++u) {
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b1[u], acc[0][1], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], acc[1][1], 0, 0, 0);
            }
        }
        // sum the wavefronts' tiles in a fixed order
        for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y)
                for (int v = 0; v < 4; ++v) red[wave][2 * x + y][v][lane] = acc[x][y][v];
        __syncthreads();
        for (int e = threadIdx.x; e < 4 * 4 * 64; e += 64 * TR_WAVES) {
            const int l = e & 63, v = (e >> 6) & 3, blk = e >> 8;
            const int x = blk >> 1, y = blk & 1;
            double sum = 0.0;
            for (int w = 0; w < TR_WAVES; ++w) sum += red[w][blk][v][l];
            const int i = i0 + 16 * x + (l >> 4) + 4 * v, c = c0 + 16 * y + (l & 15);
            if (i < J.M && c < m) {
                double* o = out + i + ldo * c;
                *o = split ? sum : J.alpha * sum + (J.beta != 0.0 ? J.beta * *o : 0.0);
            }
        }
        __syncthreads();
    }
}

// C = alpha sum_z part[z] + beta C for the jobs of a split streaming product
__global__ void stream_reduce_kernel(StreamJobs jobs, int ksplit, const double* part,
                                     long pstride) {
    const StreamJob& J = jobs.job[blockIdx.y];
    const long mn = (long)J.M * J.N;
    const double* pj = part + (long)blockIdx.y * ksplit * pstride;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < mn;
         e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e % J.M), c = (int)(e / J.M);
        double sum = 0.0;
        for (int z = 0; z < ksplit; ++z) sum += pj[z * pstride + e];
        double* o = J.C + i + J.ldc * c;
        *o = J.alpha * sum + (J.beta != 0.0 ? J.beta * *o : 0.0);
    }
}

template <int L>
static void stream_launch(int kc, const StreamJobs& jobs, int rbmax, int ksplit, double* part,
                          long pstride, hipStream_t s) {
    const dim3 grid(rbmax * ksplit, jobs.count), block(64 * TR_WAVES);
    if (kc == 128)
        hipLaunchKernelGGL((stream_kernel<L, 8>), grid, block, 0, s, jobs, ksplit, part, pstride);
    else
        hipLaunchKernelGGL((stream_kernel<L, 16>), grid, block, 0, s, jobs, ksplit, part, pstride);
}

hipError_t stream_multi(int layout, const StreamJobs& jobs, int kc, double* part, long part_cap,
                        hipStream_t s) {
    if (jobs.count <= 0) return hipSuccess;
    if (jobs.count > 3 || layout < 0 || layout > 2 || (kc != 128 && kc != 256))
        return hipErrorInvalidValue;
    int kmax = 0, rbmax = 0;
    long pmax = 0;
    for (int t = 0; t < jobs.count; ++t) {
        const StreamJob& J = jobs.job[t];
        if (J.M <= 0 || J.N <= 0 || J.K <= 0 || !J.A || !J.B || !J.C) return hipErrorInvalidValue;
        kmax = std::max(kmax, J.K);
        rbmax = std::max(rbmax, (J.M + 31) / 32);
        pmax = std::max(pmax, (long)J.M * J.N);
    }
    const int ksplit = (kmax + kc - 1) / kc;
    if (ksplit > 1 && (!part || (long)jobs.count * ksplit * pmax > part_cap))
        return hipErrorInvalidValue;   // the caller checks stream_fits first
    if (layout == 0)
        stream_launch<0>(kc, jobs, rbmax, ksplit, part, pmax, s);
    else if (layout == 1)
        stream_launch<1>(kc, jobs, rbmax, ksplit, part, pmax, s);
    else
        stream_launch<2>(kc, jobs, rbmax, ksplit, part, pmax, s);
    if (ksplit > 1) {
        const int blocks = (int)std::min<long>((pmax + 255) / 256, 1024);
        hipLaunchKernelGGL(stream_reduce_kernel, dim3(blocks, jobs.count), dim3(256), 0, s, jobs,
                           ksplit, part, pmax);
    }
    return hipGetLastError();
}

bool stream_fits(const StreamJobs& jobs, int kc, long part_cap) {
    int kmax = 0;
    long pmax = 0;
    for (int t = 0; t < jobs.count; ++t) {
        kmax = std::max(kmax, jobs.job[t].K);
        pmax = std::max(pmax, (long)jobs.job[t].M * jobs.job[t].N);
    }
    const int ksplit = (kmax + kc - 1) / kc;
    return ksplit <= 1 || (long)jobs.count * ksplit * pmax <= part_cap;
}

// dynamic LDS of the Gram-type kernels: the wavefronts' partial tiles
static size_t gram_lds(int waves) {
    return sizeof(double) * std::max((size_t)2 * 32 * GR_LD, (size_t)waves * 4 * 4 * 64);
}
template <class F>
static hipError_t set_lds_once(std::once_flag& once, hipError_t& err, F&& fns) {
    std::call_once(once, [&] {
        for (const auto& fl : fns()) {
            const hipError_t e = hipFuncSetAttribute(fl.first, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)fl.second);
            if (e != hipSuccess) err = e;
        }
    });
    return err;
}

static size_t sgram_lds(int waves, int group) {
    return sizeof(double) * std::max((size_t)2 * 32 * GR_LD + (size_t)group * GR_KC,
                                     (size_t)waves * 4 * 4 * 64);
}

// a launch of scaled-Gram batches that the grouped kernel takes: A^T diag(d_q) B
// with A and B shared by the batch
static bool sgram_fits(bool transA, bool transB, const GramJobs& jobs) {
    if (!transA || transB || jobs.count <= 0) return false;
    for (int t = 0; t < jobs.count; ++t) {
        const GemmArgs& g = jobs.g[t];
        if (!g.d || g.strideA != 0 || g.strideB != 0 || g.batch < 2 || g.inner != 1 || g.lowp)
            return false;
    }
    return true;
}

static hipError_t sgram_launch(const GramJobs& jobs, hipStream_t s, int waves, int group) {
    // (waves, terms per group): (8, 2), (8, 4), (16, 2); 16 wavefronts hold
    // at most 128 registers per lane, too few for four terms' accumulators
    if (waves == 16) group = 2;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    const void* const kern[3] = {(const void*)sgram_multi_kernel<8, 2>,
                                 (const void*)sgram_multi_kernel<8, 4>,
                                 (const void*)sgram_multi_kernel<16, 2>};
    const hipError_t ae = set_lds_once(once, attr_err, [&kern] {
        return std::vector<std::pair<const void*, size_t>>{
            {kern[0], sgram_lds(8, 2)}, {kern[1], sgram_lds(8, 4)}, {kern[2], sgram_lds(16, 2)}};
    });
    if (ae != hipSuccess) return ae;
    long blocks = 0;
    for (int t = 0; t < jobs.count; ++t) {
        const GemmArgs& g = jobs.g[t];
        if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipErrorInvalidValue;
        blocks = std::max(blocks, (long)((g.M + 31) / 32) * ((g.N + 31) / 32) *
                                      ((g.batch + group - 1) / group));
    }
    if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
    const int idx = waves == 16 ? 2 : (group == 4 ? 1 : 0);
    GramJobs j = jobs;
    void* args[] = {&j};
    return hipLaunchKernel(kern[idx], dim3((unsigned)blocks, jobs.count), dim3(64 * waves), args,
                           sgram_lds(waves, group), s);
}

// the kernel for (layout, wavefronts, staging) as a table index
static int gram_index(int L, int waves, bool staged) { return (L * 2 + (waves == 16)) * 2 + staged; }

#define FC_GRAM_TABLE(kern)                                                                        \
    {(const void*)kern<0, 8, false>, (const void*)kern<0, 8, true>, (const void*)kern<0, 16, false>, \
     (const void*)kern<0, 16, true>, (const void*)kern<1, 8, false>, (const void*)kern<1, 8, true>,   \
     (const void*)kern<1, 16, false>, (const void*)kern<1, 16, true>, (const void*)kern<2, 8, false>, \
     (const void*)kern<2, 8, true>, (const void*)kern<2, 16, false>, (const void*)kern<2, 16, true>}

static const void* const kGramKernels[12] = FC_GRAM_TABLE(gram_kernel);
static const void* const kGramMultiKernels[12] = FC_GRAM_TABLE(gram_multi_kernel);

static hipError_t gram_attrs(const void* const* table, std::once_flag& once, hipError_t& err) {
    return set_lds_once(once, err, [table] {
        std::vector<std::pair<const void*, size_t>> v;
        for (int i = 0; i < 12; ++i) v.push_back({table[i], gram_lds(((i >> 1) & 1) ? 16 : 8)});
        return v;
    });
}

hipError_t gram(bool transA, bool transB, const GemmArgs& g, hipStream_t s, int waves, bool staged,
                int group) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (g.inner != 1 || g.lowp || g.K <= 0 || (transA && transB)) return hipErrorInvalidValue;
    if (waves != 8 && waves != 16) return hipErrorInvalidValue;
    if (group != 1 && group != 2 && group != 4) return hipErrorInvalidValue;
    if (group > 1) {
        GramJobs one;
        one.count = 1;
        one.g[0] = g;
        if (sgram_fits(transA, transB, one)) return sgram_launch(one, s, waves, group);
    }
    const long tiles = (long)((g.M + 31) / 32) * ((g.N + 31) / 32);
    if (tiles > 0x7fffffffL || g.batch > 65535) return hipErrorInvalidValue;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    const hipError_t ae = gram_attrs(kGramKernels, once, attr_err);
    if (ae != hipSuccess) return ae;
    const int L = transA ? 0 : (transB ? 1 : 2);
    GemmArgs a = g;
    void* args[] = {&a};
    return hipLaunchKernel(kGramKernels[gram_index(L, waves, staged)], dim3(tiles, 1, g.batch),
                           dim3(64 * waves), args, gram_lds(waves), s);
}

hipError_t gram_multi(bool transA, bool transB, const GramJobs& jobs, hipStream_t s, int waves,
                      bool staged, int group) {
    if (jobs.count <= 0) return hipSuccess;
    if (jobs.count > kMaxGramJobs || (transA && transB) || (waves != 8 && waves != 16))
        return hipErrorInvalidValue;
    if (group != 1 && group != 2 && group != 4) return hipErrorInvalidValue;
    if (group > 1 && sgram_fits(transA, transB, jobs)) return sgram_launch(jobs, s, waves, group);
    long tiles = 0;
    for (int t = 0; t < jobs.count; ++t) {
        const GemmArgs& g = jobs.g[t];
        if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch < 1 || g.inner != 1 || g.lowp)
            return hipErrorInvalidValue;
        tiles = std::max(tiles, (long)((g.M + 31) / 32) * ((g.N + 31) / 32) * g.batch);
    }
    if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    const hipError_t ae = gram_attrs(kGramMultiKernels, once, attr_err);
    if (ae != hipSuccess) return ae;
    const int L = transA ? 0 : (transB ? 1 : 2);
    GramJobs j = jobs;
    void* args[] = {&j};
    return hipLaunchKernel(kGramMultiKernels[gram_index(L, waves, staged)],
                           dim3((unsigned)tiles, jobs.count), dim3(64 * waves), args, gram_lds(waves), s);
}

// ---------------------------------------------------------------------------
// Fused application of a separable diagonal scaling to the Tucker basis:
//   out[i, c] = sum_q sum_j Z[i, j] D[i, q] T^q[j, c]
// (i < n, c < p, j < r, q < Q; T^q the r x p block at T + q r p, ld r), i.e.
// out = sum_q diag(D[:, q]) Z T^q: a product over the reduction index (q, j)
// whose left operand, the row-wise Kronecker product Z[i, j] D[i, q], is
// formed in registers and never stored.  Tiles and reduction as in
// gram_tile: one workgroup per 32 x 32 output tile, the sixteen wavefronts
// take the terms q in turn, partial tiles summed in LDS in a fixed order.
template <int GR_WAVES>
__device__ __forceinline__ void kron_tile(int n, int Q, const KronJob& J, int tile) {
    extern __shared__ double gram_red[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tilesM = (n + 31) / 32;
    const int i0 = (tile % tilesM) * 32, c0 = (tile / tilesM) * 32;
    const int r16 = lane & 15, kq = lane >> 4;
    const int ia0 = i0 + r16, ia1 = i0 + 16 + r16;
    const int cb0 = c0 + r16, cb1 = c0 + 16 + r16;
    const bool va0 = ia0 < n, va1 = ia1 < n, vb0 = cb0 < J.p, vb1 = cb1 < J.p;
    const int r = J.r;
    const long rp = (long)r * J.p;
    const double* __restrict__ z0p = J.Z + (va0 ? ia0 : 0);
    const double* __restrict__ z1p = J.Z + (va1 ? ia1 : 0);
    const double* __restrict__ t0p = J.T + (vb0 ? (long)r * cb0 : 0);
    const double* __restrict__ t1p = J.T + (vb1 ? (long)r * cb1 : 0);
    dbl4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int steps = (r + 3) / 4;
    for (int q = wave; q < Q; q += GR_WAVES) {
        const double d0 = va0 ? J.D[ia0 + (long)n * q] : 0.0;
        const double d1 = va1 ? J.D[ia1 + (long)n * q] : 0.0;
        const double* __restrict__ tq0 = t0p + rp * q;
        const double* __restrict__ tq1 = t1p + rp * q;
        for (int s0 = 0; s0 < steps; s0 += 4) {
            double a0[4], a1[4], b0[4], b1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 4 * (s0 + u) + kq;
                const bool vk = k < r;
                a0[u] = vk ? z0p[(long)J.ldz * k] * d0 : 0.0;
                a1[u] = vk ? z1p[(long)J.ldz * k] * d1 : 0.0;
                b0[u] = (vk && vb0) ? tq0[k] : 0.0;
                b1[u] = (vk && vb1) ? tq1[k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b0[u], acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b1[u], acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b0[u], acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], acc[1][1], 0, 0, 0);
            }
        }
    }
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int v = 0; v < 4; ++v)
                gram_red[((wave * 4 + 2 * x + y) * 4 + v) * 64 + lane] = acc[x][y][v];
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * 2 * 4 * 64; e += 64 * GR_WAVES) {
        const int l = e & 63, v = (e >> 6) & 3, blk = e >> 8;
        const int x = blk >> 1, y = blk & 1;
        double sum = 0.0;
        for (int w = 0; w < GR_WAVES; ++w) sum += gram_red[((w * 4 + blk) * 4 + v) * 64 + l];
        const int i = i0 + 16 * x + (l >> 4) + 4 * v, c = c0 + 16 * y + (l & 15);
        if (i < n && c < J.p) J.out[i + J.ldo * c] = sum;
    }
}

template <int W>
__global__ __launch_bounds__(64 * W) void kron_apply_kernel(int n, int Q, KronJobs jobs) {
    const KronJob& J = jobs.job[blockIdx.y];
    const int tiles = ((n + 31) / 32) * ((J.p + 31) / 32);
    if ((int)blockIdx.x >= tiles) return;
    kron_tile<W>(n, Q, J, (int)blockIdx.x);
}

hipError_t kron_apply_multi(int n, int Q, const KronJobs& jobs, hipStream_t s, int waves) {
    if (jobs.count <= 0) return hipSuccess;
    if (jobs.count > kMaxPanelJobs || n <= 0 || Q <= 0 || (waves != 8 && waves != 16))
        return hipErrorInvalidValue;
    int tiles = 0;
    for (int t = 0; t < jobs.count; ++t) {
        const KronJob& J = jobs.job[t];
        if (J.r <= 0 || J.p <= 0 || !J.Z || !J.D || !J.T || !J.out || J.ldz < n || J.ldo < n)
            return hipErrorInvalidValue;
        tiles = std::max(tiles, ((n + 31) / 32) * ((J.p + 31) / 32));
    }
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    const hipError_t ae = set_lds_once(once, attr_err, [] {
        return std::vector<std::pair<const void*, size_t>>{
            {(const void*)kron_apply_kernel<16>, gram_lds(16)},
            {(const void*)kron_apply_kernel<8>, gram_lds(8)}};
    });
    if (ae != hipSuccess) return ae;
    if (waves == 16)
        hipLaunchKernelGGL(kron_apply_kernel<16>, dim3(tiles, jobs.count), dim3(64 * 16), gram_lds(16),
                           s, n, Q, jobs);
    else
        hipLaunchKernelGGL(kron_apply_kernel<8>, dim3(tiles, jobs.count), dim3(64 * 8), gram_lds(8), s,
                           n, Q, jobs);
    return hipGetLastError();
}

hipError_t gemm(bool transA, bool transB, const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (g.K <= 0) {
        // C = beta C
        if (g.beta == 0.0) {
            for (int b = 0; b < g.batch; ++b) {
                double* C = g.C + (long)(b / g.inner) * g.strideC + (long)(b % g.inner) * g.strideCin;
                hipError_t e = copy2d(g.M, g.N, nullptr, 0, C, g.ldc, s);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    }
    if (!transA && !transB) return gemm_dispatch<false, false>(g, s);
    if (!transA && transB) return gemm_dispatch<false, true>(g, s);
    if (transA && !transB) return gemm_dispatch<true, false>(g, s);
    return gemm_dispatch<true, true>(g, s);
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigensolver for symmetric k x k matrices (k <= 128), one
// workgroup per matrix.  The matrix lives in LDS; the accumulated rotations
// (eigenvectors) live in a global scratch matrix whose column updates are
// contiguous.  Rounds use the round-robin tournament ordering, so the k/2
// rotations of a round touch disjoint row/column pairs and run in parallel.
constexpr int JAC_THREADS = 512;

__device__ void jacobi_body(int k, const double* __restrict__ A, long lda, double* evals,
                            double* Vo_base, long ldv, double* v, double* a) {
    const int kp = k + (k & 1);
    const int half = kp / 2;
    __shared__ double cs[64], sn[64];
    __shared__ int pp[64], qq[64];
    __shared__ int nrot;
    const int tid = threadIdx.x;
    for (int e = tid; e < kp * kp; e += blockDim.x) {
        const int i = e % kp, j = e / kp;
        a[e] = (i < k && j < k) ? 0.5 * (A[i + (long)j * lda] + A[j + (long)i * lda]) : 0.0;
        v[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) nrot = 0;
        __syncthreads();
        for (int r = 0; r < kp - 1; ++r) {
            if (tid < half) {
                auto P = [&](int x) { return x == 0 ? 0 : ((x - 1 + r) % (kp - 1)) + 1; };
                int p = P(tid), q = P(kp - 1 - tid);
                if (p > q) { int t = p; p = q; q = t; }
                const double apq = a[p + q * kp];
                const double app = a[p + p * kp], aqq = a[q + q * kp];
                double c = 1.0, s = 0.0;
                if (fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * sqrt(fabs(app) * fabs(aqq))) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    atomicAdd(&nrot, 1);
                }
                cs[tid] = c; sn[tid] = s; pp[tid] = p; qq[tid] = q;
            }
            __syncthreads();
            for (int e = tid; e < half * kp; e += blockDim.x) {
                const int i = e / kp, j = e % kp;
                const double c = cs[i], s = sn[i];
                if (s == 0.0) continue;
                const int p = pp[i], q = qq[i];
                const double x = a[p + j * kp], y = a[q + j * kp];
                a[p + j * kp] = c * x - s * y;
                a[q + j * kp] = s * x + c * y;
            }
            __syncthreads();
            for (int e = tid; e < half * kp; e += blockDim.x) {
                const int i = e / kp, j = e % kp;
                const double c = cs[i], s = sn[i];
                if (s == 0.0) continue;
                const int p = pp[i], q = qq[i];
                const double x = a[j + p * kp], y = a[j + q * kp];
                a[j + p * kp] = c * x - s * y;
                a[j + q * kp] = s * x + c * y;
                const double vx = v[j + p * kp], vy = v[j + q * kp];
                v[j + p * kp] = c * vx - s * vy;
                v[j + q * kp] = s * vx + c * vy;
            }
            __syncthreads();
        }
        if (nrot == 0) break;
        __syncthreads();
    }
    for (int i = tid; i < k; i += blockDim.x) {
        const double ei = a[i + i * kp];
        int rank = 0;
        for (int j = 0; j < k; ++j) {
            const double ej = a[j + j * kp];
            if (ej > ei || (ej == ei && j < i)) ++rank;
        }
        evals[rank] = ei;
        double* Vo = Vo_base + (long)rank * ldv;
        for (int j = 0; j < k; ++j) Vo[j] = v[j + i * kp];
    }
}

__global__ __launch_bounds__(JAC_THREADS) void jacobi_kernel(int k, const double* __restrict__ Ain,
                                                             long lda, long strideA, double* evals,
                                                             double* Vout, long ldv, long strideV,
                                                             double* scratch) {
    extern __shared__ double sm[];
    const int kp = k + (k & 1);
    const int b = blockIdx.x;
    jacobi_body(k, Ain + (long)b * strideA, lda, evals + (long)b * k, Vout + (long)b * strideV, ldv,
                scratch + (long)b * kp * kp, sm);
}


// ---------------------------------------------------------------------------
// Dense symmetric eigensolver for k <= 128, one workgroup per matrix:
//  1. Householder reduction to tridiagonal form in LDS (reflectors kept in
//     the lower triangle), four barriers per step;
//  2. eigenvalues by multisection on Sturm counts: four lanes per
//     eigenvalue, eight points per step;
//  3. eigenvectors of the tridiagonal matrix by inverse iteration with a
//     partially pivoted tridiagonal LU, one vector per thread (factors in a
//     coalesced global scratch);
//  4. the eigenvectors move to LDS (one padded column each; the reflectors
//     to global scratch) and vectors of clusters of close eigenvalues are
//     re-orthogonalised against all their predecessors;
//  5. back-transformation: each wavefront applies all reflectors to the
//     columns it owns, with no barrier between reflectors.
// The Sturm recurrence divides by a Newton-refined hardware reciprocal, and
// the LU factors keep reciprocal pivots, so neither inner loop runs the full
// division sequence.
// Eigenvalues are returned in descending order.  Eigenvectors belonging to
// eigenvalues at most 1e-17 of the largest in magnitude are neither refined
// nor back-transformed (callers do not use them).  Scratch: 6 k^2 doubles.
constexpr int TD_THREADS = 512;
constexpr int TRI_THREADS = 1024;   // the tridiagonalisation's workgroup
constexpr int TRI_PARTS = TRI_THREADS / 128;   // column groups of its matrix-vector step

__device__ inline double td_wave_sum(double v) { return wave_sum(v); }

// 1/q for the Sturm recurrence: the hardware reciprocal estimate refined by
// two Newton steps (r <- r + r (1 - q r)), accurate to a few ulp; |q| is
// kept at or above the pivot floor, so no operand scaling is needed
__device__ inline double td_recip(double q) {
    double r = __builtin_amdgcn_rcp(q);
    double t = fma(-q, r, 1.0);
    r = fma(r, t, r);
    t = fma(-q, r, 1.0);
    return fma(r, t, r);
}

// Scratch layout of one job (6 k^2 doubles): reflectors R (k x k, the lower
// triangle of the reduced matrix), the eigenvectors X of the tridiagonal
// matrix (element j of vector i at X[i + j k]), d, e, tau, the eigenvalues
// (descending) and the number of vectors wanted.
#define TD_X(k) ((long)(k) * (k))
#define TD_D(k) (2L * (k) * (k))
#define TD_E(k) (TD_D(k) + (k))
#define TD_TAU(k) (TD_D(k) + 2L * (k))
#define TD_LAM(k) (TD_D(k) + 3L * (k))
#define TD_NV(k) (TD_D(k) + 4L * (k))
#define TD_BND(k) (TD_NV(k) + 1)   // Gershgorin lo, hi and max(|lo|, |hi|) of (d, e)

__global__ __launch_bounds__(TRI_THREADS) void tdeig_tri_kernel(EigJobs jobs) {
    extern __shared__ double sm[];
    __shared__ double sc[2];
    const EigJob& J = jobs.job[blockIdx.x];
    const int k = J.k;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int kp = k + 1;            // padded leading dimension of the eigenvector block
    double* a = sm;                  // phase 1: the matrix (ld k); phases 4-5: eigenvectors (ld kp)
    double* d = sm + (long)k * kp;   // diagonal
    double* e = d + k;               // off-diagonal
    double* tau = e + k;             // reflector scalars
    double* vv = tau + k;            // current reflector
    double* pw = vv + k;             // p / w / dot products
    double* lam = pw + k;            // eigenvalues, descending
    double* e2 = lam + k;            // squared off-diagonal
    double* pw4 = e2 + k;            // partial sums of A22 v (TRI_PARTS x 128)
    // the symmetrised matrix into LDS, eight elements per thread in flight
    for (int x0 = 0; x0 < k * k; x0 += 8 * TRI_THREADS) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = x0 + tid + u * TRI_THREADS;
            const int i = x % k, j = x / k;
            v[u] = x < k * k ? 0.5 * (J.A[i + (long)j * J.lda] + J.A[j + (long)i * J.lda]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = x0 + tid + u * TRI_THREADS;
            if (x < k * k) a[x] = v[u];
        }
    }
    __syncthreads();
    if (k == 1) {
        if (tid == 0) { J.evals[0] = a[0]; J.V[0] = 1.0; }
        return;
    }
    if (blockIdx.x >= (unsigned)jobs.count) return;
    // 1. tridiagonalisation; the first wavefront forms each reflector and the
    //    scalar products, so a step costs four barriers
    for (int j = 0; j + 2 < k; ++j) {
        const int m = k - j - 1;
        if (wv == 0) {
            double s = 0.0;
            for (int r = lane; r < m; r += 64) { const double x = a[(j + 1 + r) + j * k]; s += x * x; }
            const double nrm2 = td_wave_sum(s);
            const double x0 = a[(j + 1) + j * k];
            const double sub = sqrt(nrm2 - x0 * x0 > 0 ? nrm2 - x0 * x0 : 0.0);
            if (sub == 0.0) {
                if (lane == 0) { d[j] = a[j + j * k]; e[j] = x0; tau[j] = 0.0; sc[j & 1] = 0.0; }
            } else {
                const double alpha = x0 > 0 ? -sqrt(nrm2) : sqrt(nrm2);
                const double v0 = x0 - alpha;
                for (int r = lane; r < m; r += 64) {
                    const double v = (r == 0) ? 1.0 : a[(j + 1 + r) + j * k] / v0;
                    vv[r] = v;
                    a[(j + 1 + r) + j * k] = v;     // keep the reflector
                }
                if (lane == 0) { d[j] = a[j + j * k]; e[j] = alpha; tau[j] = -v0 / alpha; sc[j & 1] = -v0 / alpha; }
            }
        }
        __syncthreads();
        const double t = sc[j & 1];
        if (t == 0.0) continue;
        // p = t * A22 v: thread (row r = tid % 128, part = tid / 128) sums over
        // the columns c = part, part + TRI_PARTS, ..., so a wavefront reads 64
        // consecutive rows of one column (no LDS bank conflicts); the first
        // wavefront adds the partial sums of each row in a fixed order
        {
            const int r = tid & 127, part = tid >> 7;
            double acc = 0.0;
            if (r < m)
                for (int c = part; c < m; c += TRI_PARTS) acc += a[(j + 1 + r) + (j + 1 + c) * k] * vv[c];
            pw4[part * 128 + r] = acc;
        }
        __syncthreads();
        if (wv == 0) {
            double sp = 0.0;
            for (int r = lane; r < m; r += 64) {
                double s8 = 0.0;
#pragma unroll
                for (int q = 0; q < TRI_PARTS; q += 2) s8 += pw4[q * 128 + r] + pw4[(q + 1) * 128 + r];
                const double pr = t * s8;
                pw[r] = pr;
                sp += vv[r] * pr;
            }
            const double K = 0.5 * t * td_wave_sum(sp);
            for (int r = lane; r < m; r += 64) pw[r] -= K * vv[r];
        }
        __syncthreads();
        if (m > 64) {
            // lane l updates rows l and l+64 (k <= 128), wavefront w columns
            // w, w+8, ...: the row factors stay in registers
            const bool in1 = lane + 64 < m;
            const double vr0 = vv[lane], wr0 = pw[lane];
            const double vr1 = in1 ? vv[lane + 64] : 0.0, wr1 = in1 ? pw[lane + 64] : 0.0;
            for (int c = wv; c < m; c += TRI_THREADS / 64) {
                const double vc = vv[c], wc = pw[c];
                double* col = a + (j + 1) + (long)(j + 1 + c) * k;
                col[lane] -= vr0 * wc + wr0 * vc;
                if (in1) col[lane + 64] -= vr1 * wc + wr1 * vc;
            }
        } else {
            for (int x = tid; x < m * m; x += blockDim.x) {
                const int r = x % m, c = x / m;
                a[(j + 1 + r) + (j + 1 + c) * k] -= vv[r] * pw[c] + pw[r] * vv[c];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        d[k - 2] = a[(k - 2) + (k - 2) * k];
        d[k - 1] = a[(k - 1) + (k - 1) * k];
        e[k - 2] = a[(k - 1) + (k - 2) * k];
        tau[k - 2] = 0.0;
    }
    __syncthreads();
    for (int i = tid; i + 1 < k; i += blockDim.x) e2[i] = e[i] * e[i];
    __syncthreads();
    // hand the reflectors (lower triangle of a), d, e and tau to the next phases
    double* S = J.scratch;
    if (tid < 64) {
        // Gershgorin bounds: min and max over the rows, two rows per lane
        // (exact operations, so any order gives the same values)
        double lo = INFINITY, hi = -INFINITY;
        for (int i = tid; i < k; i += 64) {
            const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < k ? fabs(e[i]) : 0.0);
            lo = fmin(lo, d[i] - r);
            hi = fmax(hi, d[i] + r);
        }
        for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off, 64));
            hi = fmax(hi, __shfl_xor(hi, off, 64));
        }
        if (tid == 0) {
            S[TD_BND(k)] = lo;
            S[TD_BND(k) + 1] = hi;
            S[TD_BND(k) + 2] = fmax(fabs(lo), fabs(hi));
        }
    }
    for (int x = tid; x < k * k; x += blockDim.x) S[x] = a[x];
    for (int i = tid; i < k; i += blockDim.x) {
        S[TD_D(k) + i] = d[i];
        S[TD_E(k) + i] = e[i];
        S[TD_TAU(k) + i] = tau[i];
    }
}

// 2. Eigenvalues by multisection on Sturm counts: one wavefront per
//    eigenvalue, its 64 lanes counting at 64 interior points of the bracket,
//    so every step shrinks the bracket 65-fold (10 steps: 65^-10 < 1e-18 of
//    2 |T|).  Eight eigenvalues per workgroup, the workgroups of all jobs in
//    one launch.
__global__ __launch_bounds__(TD_THREADS) void tdeig_val_kernel(EigJobs jobs) {
    __shared__ double d[128], e2[128], sb[4];
    const EigJob& J = jobs.job[blockIdx.y];
    const int k = J.k;
    if (k <= 1 || (int)blockIdx.x * (TD_THREADS / 64) >= k) return;
    const double* S = J.scratch;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i < k; i += blockDim.x) {
        d[i] = S[TD_D(k) + i];
        const double ee = S[TD_E(k) + i];
        e2[i] = (i + 1 < k) ? ee * ee : 0.0;
    }
    if (tid < 3) sb[tid] = S[TD_BND(k) + tid];
    __syncthreads();
    const int grp = blockIdx.x * (TD_THREADS / 64) + wv;
    if (grp >= k) return;
    const double tnorm = sb[2];
    const double pivmin = fmax(1e-300, 1e-30 * tnorm * tnorm);
    const int want = k - 1 - grp;   // number of eigenvalues below the target
    double l = sb[0] - 1e-14 * tnorm - 1e-300, h = sb[1] + 1e-14 * tnorm + 1e-300;
    for (int it = 0; it < 10; ++it) {
        const double w = (h - l) / 65.0;
        const double x = l + w * (lane + 1);
        double q = d[0] - x;
        if (fabs(q) < pivmin) q = -pivmin;
        int c = q < 0;
        for (int i = 1; i < k; ++i) {
            q = (d[i] - x) - e2[i - 1] * td_recip(q);
            if (fabs(q) < pivmin) q = -pivmin;
            c += q < 0;
        }
        // counts are monotone in x: the first z points have at most `want`
        // eigenvalues below them
        const int z = __popcll(__ballot(c <= want));
        const double nl = l + w * z;
        const double nh = (z == 64) ? h : l + w * (z + 1);
        l = nl;
        h = nh;
    }
    if (lane == 0) J.scratch[TD_LAM(k) + grp] = 0.5 * (l + h);
}

// the rank rule of the truncations on the eigenvalues (descending): the
// number of eigenvectors wanted
__device__ inline int td_nvec(const EigJob& J, const double* lam) {
    const int k = J.k;
    if (J.budget < 0.0) return k;
    double tail = 0.0;
    int rr = k;
    for (int i = k - 1; i >= 0; --i) {
        tail += fmax(lam[i], 0.0);
        if (tail <= J.budget) rr = i; else break;
    }
    int numrank = 0;
    const double tmax = fmax(lam[0], 0.0);
    while (numrank < k && lam[numrank] > 1e-17 * tmax) ++numrank;
    return min(min(max(numrank, 1), max(rr + J.margin, 1)), k);
}

// 3. Eigenvectors of the tridiagonal matrix by inverse iteration with a
//    partially pivoted LU (reciprocal pivots), one vector per thread,
//    TD_VPB vectors per workgroup, the factors and the iterate in LDS.
constexpr int TD_VPB = 16;
__global__ __launch_bounds__(64) void tdeig_vec_kernel(EigJobs jobs) {
    extern __shared__ double lu[];
    __shared__ double dd[128], ee[128], lams[128], sb[2];
    __shared__ int nv_s;
    const EigJob& J = jobs.job[blockIdx.y];
    const int k = J.k;
    if (k <= 1 || (int)blockIdx.x * TD_VPB >= k) return;
    double* S = J.scratch;
    const int tid = threadIdx.x;
    for (int i = tid; i < k; i += blockDim.x) {
        dd[i] = S[TD_D(k) + i];
        ee[i] = S[TD_E(k) + i];
        lams[i] = S[TD_LAM(k) + i];
    }
    if (tid == 0) sb[0] = S[TD_BND(k) + 2];
    __syncthreads();
    if (tid == 0) {
        // the rank rule's scan runs on the LDS copy of the eigenvalues
        const int nv = td_nvec(J, lams);
        nv_s = nv;
        if (blockIdx.x == 0) S[TD_NV(k)] = (double)nv;
    }
    __syncthreads();
    const int i = blockIdx.x * TD_VPB + tid;
    if (tid >= TD_VPB || i >= nv_s) return;
    const double tnorm = sb[0];
    const double smallpiv = 1e-15 * fmax(tnorm, 1e-300);
    // LDS arrays [j][TD_VPB]: U0 (reciprocal pivots), U1, U2, ML (multipliers),
    // SW (row interchange), X (iterate)
    double* U0 = lu;
    double* U1 = U0 + k * TD_VPB;
    double* U2 = U1 + k * TD_VPB;
    double* ML = U2 + k * TD_VPB;
    double* SW = ML + k * TD_VPB;
    double* X = SW + k * TD_VPB;
#define TDV(A, j) A[(j) * TD_VPB + tid]
    const double lm = S[TD_LAM(k) + i] + 4e-16 * tnorm * (1 + (i % 3));
    // factor T - lm I (rows: sub c_j = e[j-1], diag, super e[j])
    double ad = dd[0] - lm, bd = (k > 1) ? ee[0] : 0.0, fd = 0.0;
    for (int j = 0; j + 1 < k; ++j) {
        const double c = ee[j];
        const double an = dd[j + 1] - lm;
        const double bn = (j + 2 < k) ? ee[j + 1] : 0.0;
        if (fabs(ad) >= fabs(c)) {
            const double mlt = (ad != 0.0) ? c / ad : 0.0;
            TDV(U0, j) = 1.0 / ((fabs(ad) < smallpiv) ? copysign(smallpiv, ad) : ad);
            TDV(U1, j) = bd;
            TDV(U2, j) = fd;
            TDV(ML, j) = mlt;
            TDV(SW, j) = 0.0;
            ad = an - mlt * bd;
            bd = bn - mlt * fd;
            fd = 0.0;
        } else {
            const double mlt = ad / c;
            TDV(U0, j) = 1.0 / c;
            TDV(U1, j) = an;
            TDV(U2, j) = bn;
            TDV(ML, j) = mlt;
            TDV(SW, j) = 1.0;
            const double na = bd - mlt * an;
            const double nb = fd - mlt * bn;
            ad = na;
            bd = nb;
            fd = 0.0;
        }
    }
    TDV(U0, k - 1) = 1.0 / ((fabs(ad) < smallpiv) ? copysign(smallpiv, ad) : ad);
    TDV(U1, k - 1) = 0.0;
    TDV(U2, k - 1) = 0.0;
    for (int j = 0; j < k; ++j) TDV(X, j) = 1.0 + 0.37 * ((j * 7 + i * 13) % 11) / 11.0;
    for (int it = 0; it < 3; ++it) {
        // forward: the row operations on the right-hand side
        double carry = TDV(X, 0);
        for (int j = 0; j + 1 < k; ++j) {
            double r0 = carry, r1 = TDV(X, j + 1);
            if (TDV(SW, j) != 0.0) { const double t2 = r0; r0 = r1; r1 = t2; }
            r1 -= TDV(ML, j) * r0;
            TDV(X, j) = r0;
            carry = r1;
        }
        TDV(X, k - 1) = carry;
        // back substitution
        double x1 = 0.0, x2 = 0.0, nrm = 0.0;
        for (int j = k - 1; j >= 0; --j) {
            const double v = (TDV(X, j) - TDV(U1, j) * x1 - TDV(U2, j) * x2) * TDV(U0, j);
            TDV(X, j) = v;
            x2 = x1;
            x1 = v;
            nrm += v * v;
        }
        const double inv = nrm > 0 ? 1.0 / sqrt(nrm) : 0.0;
        for (int j = 0; j < k; ++j) TDV(X, j) *= inv;
    }
    for (int j = 0; j < k; ++j) S[TD_X(k) + i + (long)j * k] = TDV(X, j);
#undef TDV
}

// 4. Vectors of clusters of close eigenvalues (descending order) are
//    re-orthogonalised against ALL their predecessors: inverse iteration
//    returns nearly parallel vectors inside a cluster, and normalising what
//    is left after removing the cluster alone would magnify their rounding
//    components along the other eigenvectors.  Dot products one wavefront
//    per predecessor, one subtraction sweep, two passes, then normalise.
//    Vectors of eigenvalues at most 1e-17 of the largest in magnitude are
//    not refined (callers never use them) and are skipped as predecessors.
//    One workgroup per matrix; it returns at once when there is no cluster.
__global__ __launch_bounds__(TD_THREADS) void tdeig_clu_kernel(EigJobs jobs) {
    extern __shared__ double sm[];
    __shared__ int any_s;
    const EigJob& J = jobs.job[blockIdx.x];
    const int k = J.k;
    if (k <= 1) return;
    double* S = J.scratch;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int kp = k + 1;
    const double* lam = S + TD_LAM(k);
    const int nvec = (int)S[TD_NV(k)];
    const double lmax = fmax(fabs(lam[0]), fabs(lam[k - 1]));
    if (tid == 0) any_s = 0;
    __syncthreads();
    for (int i = 1 + tid; i < nvec; i += blockDim.x)
        if (fabs(lam[i]) > 1e-17 * lmax && lam[i - 1] - lam[i] < 1e-9 * lmax) any_s = 1;
    __syncthreads();
    if (!any_s) return;
    double* Xl = sm;                      // vector i at Xl + i kp
    double* pw = sm + (long)k * kp;       // dot products
    double* used = pw + k;                // 1 for a vector that is refined
    double* X = S + TD_X(k);
    for (int x0 = 0; x0 < nvec * k; x0 += 8 * TD_THREADS) {   // eight loads in flight
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = x0 + tid + u * TD_THREADS;
            const int i = x % nvec, j = x / nvec;
            v[u] = x < nvec * k ? X[i + (long)j * k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = x0 + tid + u * TD_THREADS;
            const int i = x % nvec, j = x / nvec;
            if (x < nvec * k) Xl[j + (long)i * kp] = v[u];
        }
    }
    for (int i = tid; i < k; i += blockDim.x) used[i] = fabs(lam[i]) > 1e-17 * lmax ? 1.0 : 0.0;
    __syncthreads();
    for (int i = 1; i < nvec; ++i) {
        if (used[i] == 0.0 || lam[i - 1] - lam[i] >= 1e-9 * lmax) continue;
        double* xi = Xl + (long)i * kp;
        for (int pass = 0; pass < 2; ++pass) {
            for (int c = wv; c < i; c += TD_THREADS / 64) {
                const double* xc = Xl + (long)c * kp;
                double acc = 0.0;
                for (int r = lane; r < k; r += 64) acc += xc[r] * xi[r];
                acc = td_wave_sum(acc);
                if (lane == 0) pw[c] = acc * used[c];
            }
            __syncthreads();
            // four threads per row, each over a quarter of the predecessors
            for (int base = 0; base < 4 * k; base += blockDim.x) {
                const int x = base + tid;
                const int r = x >> 2, part = x & 3;
                double acc = 0.0;
                if (r < k)
                    for (int c = part; c < i; c += 4) acc += pw[c] * Xl[r + (long)c * kp];
                acc += __shfl_xor(acc, 1, 64);
                acc += __shfl_xor(acc, 2, 64);
                if (r < k && part == 0) xi[r] -= acc;
            }
            __syncthreads();
        }
        if (wv == 0) {
            double s3 = 0.0;
            for (int r = lane; r < k; r += 64) s3 += xi[r] * xi[r];
            const double nn = sqrt(td_wave_sum(s3));
            const double f = nn > 0 ? 1.0 / nn : 0.0;
            for (int r = lane; r < k; r += 64) xi[r] *= f;
        }
        __syncthreads();
    }
    for (int x = tid; x < nvec * k; x += blockDim.x) {
        const int i = x % nvec, j = x / nvec;
        X[i + (long)j * k] = Xl[j + (long)i * kp];
    }
}

// 5. Back-transformation V = H_0 ... H_{k-3} X (reflector j acts on rows
//    j+1..k-1): one wavefront per eigenvector, lane l holding rows l and
//    l + 64 of the vector and of each reflector (read from scratch one
//    reflector ahead), eight vectors per workgroup, all jobs in one launch.
//    Vectors of eigenvalues at most 1e-17 of the largest in magnitude are
//    written as they are.  The first workgroup of a job writes its
//    eigenvalues.
__global__ __launch_bounds__(TD_THREADS) void tdeig_back_kernel(EigJobs jobs) {
    const EigJob& J = jobs.job[blockIdx.y];
    const int k = J.k;
    if (k <= 1) return;
    const double* S = J.scratch;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double* lam = S + TD_LAM(k);
    if (blockIdx.x == 0)
        for (int i = tid; i < k; i += blockDim.x) J.evals[i] = lam[i];
    const int nvec = (int)S[TD_NV(k)];
    const int i = blockIdx.x * (TD_THREADS / 64) + wv;
    if (i >= nvec) return;
    const double lmax = fmax(fabs(lam[0]), fabs(lam[k - 1]));
    const double* X = S + TD_X(k);
    const int r0 = lane, r1 = lane + 64;
    double x0 = r0 < k ? X[i + (long)r0 * k] : 0.0;
    double x1 = r1 < k ? X[i + (long)r1 * k] : 0.0;
    if (fabs(lam[i]) > 1e-17 * lmax) {
        const double* R = S;   // reflector j: R[rho + j k], rho > j
        auto refl = [&](int jj, int rho) { return (rho > jj && rho < k) ? R[rho + (long)jj * k] : 0.0; };
        double c0 = 0.0, c1 = 0.0;
        if (k >= 3) { c0 = refl(k - 3, r0); c1 = refl(k - 3, r1); }
        for (int j = k - 3; j >= 0; --j) {
            double n0 = 0.0, n1 = 0.0;
            if (j > 0) { n0 = refl(j - 1, r0); n1 = refl(j - 1, r1); }
            const double t = S[TD_TAU(k) + j];
            if (t != 0.0) {
                const double sj = t * td_wave_sum(c0 * x0 + c1 * x1);
                x0 -= sj * c0;
                x1 -= sj * c1;
            }
            c0 = n0;
            c1 = n1;
        }
    }
    if (r0 < k) J.V[r0 + (long)i * J.ldv] = x0;
    if (r1 < k) J.V[r1 + (long)i * J.ldv] = x1;
}

hipError_t sym_eig_multi(const EigJobs& jobs, hipStream_t s) {
    int kmax = 0;
    for (int i = 0; i < jobs.count; ++i) {
        if (jobs.job[i].k > 128) return hipErrorInvalidValue;
        kmax = std::max(kmax, jobs.job[i].k);
    }
    if (jobs.count <= 0 || kmax <= 0) return hipSuccess;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] {
        hipError_t e = hipFuncSetAttribute((const void*)tdeig_tri_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)tdeig_clu_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)tdeig_vec_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 100 * 1024);
        attr_err = e;
    });
    if (attr_err != hipSuccess) return attr_err;
    const int per = TD_THREADS / 64;
    static_assert(TRI_THREADS % 128 == 0 && TRI_PARTS % 2 == 0,
                  "the tridiagonalisation's matrix-vector step takes whole groups of 128 threads");
    hipLaunchKernelGGL(tdeig_tri_kernel, dim3(jobs.count), dim3(TRI_THREADS),
                       sizeof(double) * ((size_t)kmax * (kmax + 1) + 7 * kmax + 128 * TRI_PARTS), s, jobs);
    hipLaunchKernelGGL(tdeig_val_kernel, dim3((kmax + per - 1) / per, jobs.count),
                       dim3(TD_THREADS), 0, s, jobs);
    hipLaunchKernelGGL(tdeig_vec_kernel, dim3((kmax + TD_VPB - 1) / TD_VPB, jobs.count), dim3(64),
                       sizeof(double) * 6 * (size_t)kmax * TD_VPB, s, jobs);
    hipLaunchKernelGGL(tdeig_clu_kernel, dim3(jobs.count), dim3(TD_THREADS),
                       sizeof(double) * ((size_t)kmax * (kmax + 1) + 2 * kmax), s, jobs);
    hipLaunchKernelGGL(tdeig_back_kernel, dim3((kmax + per - 1) / per, jobs.count),
                       dim3(TD_THREADS), 0, s, jobs);
    return hipGetLastError();
}

hipError_t sym_eig(int k, int batch, const double* A, long lda, long strideA, double* evals,
                   double* V, long ldv, long strideV, double* scratch, hipStream_t s) {
    if (k <= 0 || batch <= 0) return hipSuccess;
    if (k > 128) return hipErrorInvalidValue;
    const int kp = k + (k & 1);
    const size_t shm = sizeof(double) * kp * kp;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] {
        attr_err = hipFuncSetAttribute((const void*)jacobi_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024);
    });
    if (attr_err != hipSuccess) return attr_err;
    hipLaunchKernelGGL(jacobi_kernel, dim3(batch), dim3(JAC_THREADS), shm, s, k, A, lda, strideA,
                       evals, V, ldv, strideV, scratch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tucker-to-canonical term selection (Appendix 1, the T2C step).  The
// candidate terms are the (slice nu, singular value j) pairs of the mode-3
// slices of an all-orthogonal core, with energies sig2[nu * r1 + j]
// (negative rounding clamped to 0).  Ordered by (energy, nu, j) ascending,
// the smallest are dropped while the cumulative dropped energy stays within
// budget2; the kept ones go to keep[t], t < K, in descending order, and K to
// *count.  One workgroup: a bitonic sort of (energy bits, index) pairs (the
// bit pattern of a non-negative double orders like its value), in LDS up to
// kT2cLds terms and in `scratch` beyond, then a block scan of the sorted
// energies in a fixed order.
constexpr int T2C_THREADS = 1024;
constexpr int kT2cLds = 8192;

__global__ __launch_bounds__(T2C_THREADS) void t2c_select_kernel(int N, int Np,
                                                                 const double* __restrict__ sig2,
                                                                 double budget2,
                                                                 unsigned long long* gkey,
                                                                 unsigned* gidx, int* keep,
                                                                 int* count) {
    extern __shared__ unsigned long long t2c_lds[];
    __shared__ double part[T2C_THREADS];
    __shared__ int cnt[T2C_THREADS];
    const int tid = threadIdx.x;
    unsigned long long* key = gkey ? gkey : t2c_lds;
    unsigned* idx = gidx ? gidx : (unsigned*)(t2c_lds + Np);
    for (int i = tid; i < Np; i += T2C_THREADS) {
        if (i < N) {
            const double v = sig2[i] > 0.0 ? sig2[i] : 0.0;
            key[i] = (unsigned long long)__double_as_longlong(v);
            idx[i] = (unsigned)i;
        } else {
            key[i] = ~0ULL;
            idx[i] = 0xffffffffu;
        }
    }
    __syncthreads();
    for (int k = 2; k <= Np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < Np; i += T2C_THREADS) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const bool gt = key[i] > key[l] || (key[i] == key[l] && idx[i] > idx[l]);
                    if (gt == up) {
                        const unsigned long long tk = key[i];
                        key[i] = key[l];
                        key[l] = tk;
                        const unsigned ti = idx[i];
                        idx[i] = idx[l];
                        idx[l] = ti;
                    }
                }
            }
            __syncthreads();
        }
    }
    // inclusive prefix sums of the sorted energies: contiguous chunks per
    // thread, then a scan of the chunk sums; count the prefixes within budget
    const int chunk = (N + T2C_THREADS - 1) / T2C_THREADS;
    const int b0 = min(N, tid * chunk), b1 = min(N, b0 + chunk);
    double loc = 0.0;
    for (int i = b0; i < b1; ++i) loc += __longlong_as_double((long long)key[i]);
    part[tid] = loc;
    __syncthreads();
    for (int off = 1; off < T2C_THREADS; off <<= 1) {
        const double add = tid >= off ? part[tid - off] : 0.0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    double run = tid > 0 ? part[tid - 1] : 0.0;
    int dropped = 0;
    for (int i = b0; i < b1; ++i) {
        run += __longlong_as_double((long long)key[i]);
        if (run <= budget2) ++dropped;
    }
    cnt[tid] = dropped;
    __syncthreads();
    for (int off = T2C_THREADS / 2; off > 0; off >>= 1) {
        if (tid < off) cnt[tid] += cnt[tid + off];
        __syncthreads();
    }
    const int K = N - cnt[0];
    for (int t = tid; t < K; t += T2C_THREADS) keep[t] = (int)idx[N - 1 - t];
    if (tid == 0) *count = K;
}

hipError_t t2c_select(int N, const double* sig2, double budget2, void* scratch, int* keep,
                      int* count, hipStream_t s) {
    if (N <= 0 || N > kT2cMaxTerms) return hipErrorInvalidValue;
    int Np = 1;
    while (Np < N) Np <<= 1;
    size_t lds = 0;
    unsigned long long* gkey = nullptr;
    unsigned* gidx = nullptr;
    if (Np <= kT2cLds) {
        lds = (sizeof(unsigned long long) + sizeof(unsigned)) * (size_t)Np;
    } else {
        gkey = (unsigned long long*)scratch;
        gidx = (unsigned*)(gkey + Np);
    }
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] {
        attr_err = hipFuncSetAttribute((const void*)t2c_select_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((sizeof(unsigned long long) + sizeof(unsigned)) * kT2cLds));
    });
    if (attr_err != hipSuccess) return attr_err;
    hipLaunchKernelGGL(t2c_select_kernel, dim3(1), dim3(T2C_THREADS), lds, s, N, Np, sig2, budget2,
                       gkey, gidx, keep, count);
    return hipGetLastError();
}

// Canonical factors of the kept T2C terms: for term t = (nu, j), with v the
// j-th eigenvector of the nu-th slice Gram (column j of the r1 x r1 block
// at V + nu r1 r1), g = core[:, :, nu] v; c0[:, t] = g / |g|, c1[:, t] = v,
// c2[:, t] = e_nu, w[t] = |g| (or the singular value when g vanishes).  One
// wavefront per term.
__global__ __launch_bounds__(256) void t2c_coef_kernel(int r0, int r1, int r2, int K,
                                                       const double* __restrict__ core,
                                                       const double* __restrict__ V,
                                                       const double* __restrict__ ev,
                                                       const int* __restrict__ keep,
                                                       double* __restrict__ c0,
                                                       double* __restrict__ c1,
                                                       double* __restrict__ c2,
                                                       double* __restrict__ w) {
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= K) return;
    const int e = keep[t];
    const int nu = e / r1, j = e % r1;
    const double* v = V + (long)nu * r1 * r1 + (long)j * r1;
    const double* cs = core + (long)r0 * r1 * nu;
    double g[2] = {0.0, 0.0};
    for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        if (i < r0) {
            double acc = 0.0;
            for (int jj = 0; jj < r1; ++jj) acc += cs[i + (long)r0 * jj] * v[jj];
            g[h] = acc;
        }
    }
    const double nrm = sqrt(wave_sum(g[0] * g[0] + g[1] * g[1]));
    for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        if (i < r0) c0[(long)t * r0 + i] = nrm > 0.0 ? g[h] / nrm : 0.0;
    }
    for (int jj = lane; jj < r1; jj += 64) c1[(long)t * r1 + jj] = v[jj];
    for (int q = lane; q < r2; q += 64) c2[(long)t * r2 + q] = q == nu ? 1.0 : 0.0;
    if (lane == 0) {
        const double s2 = ev[e] > 0.0 ? ev[e] : 0.0;
        w[t] = nrm > 0.0 ? nrm : sqrt(s2);
    }
}

hipError_t t2c_coef(int r0, int r1, int r2, int K, const double* core, const double* V,
                    const double* ev, const int* keep, double* c0, double* c1, double* c2,
                    double* w, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    if (r0 > 128 || r0 <= 0 || r1 <= 0 || r2 <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(t2c_coef_kernel, dim3((K + 3) / 4), dim3(256), 0, s, r0, r1, r2, K, core, V,
                       ev, keep, c0, c1, c2, w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Probe sums of the projection check of the Hadamard truncation: for two
// problems (blockIdx.y) and S probes (blockIdx.x),
//   out[2 t + y] = sum_q sum_k U2_t[k, q] sum_j M_t[j + r1 k + r1 r2 q] U1_t[j, q]
// (M_t at M + t mstride; U1_t r1 x Q at U1 + t r1 Q; U2_t r2 x Q at U2 + t r2 Q).
// Wavefronts take the (q, k) pairs in turn, lanes the index j (r1 <= 128);
// the lane sums are added in a fixed order at the end.
constexpr int PB_THREADS = 1024;
__global__ __launch_bounds__(PB_THREADS) void probe_sum_kernel(ProbeSums a) {
    __shared__ double red[PB_THREADS / 64];
    const ProbeSum& P = a.p[blockIdx.y];
    const int t = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long rr = (long)P.r1 * P.r2;
    const double* M = P.M + (long)t * P.mstride;
    const double* U1 = P.U1 + (long)t * P.r1 * P.Q;
    const double* U2 = P.U2 + (long)t * P.r2 * P.Q;
    double acc = 0.0;
    for (long qk = wave; qk < (long)P.r2 * P.Q; qk += PB_THREADS / 64) {
        const int k = (int)(qk % P.r2), q = (int)(qk / P.r2);
        const double u2 = U2[k + (long)P.r2 * q];
        const double* Mc = M + (long)P.r1 * k + rr * q;
        const double* u1 = U1 + (long)P.r1 * q;
        for (int j = lane; j < P.r1; j += 64) acc += u2 * Mc[j] * u1[j];
    }
    acc = wave_sum(acc);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < PB_THREADS / 64; ++w) sum += red[w];
        a.out[2 * t + blockIdx.y] = sum;
    }
}

hipError_t probe_sums(const ProbeSums& a, int S, hipStream_t s) {
    if (S <= 0) return hipSuccess;
    for (int y = 0; y < 2; ++y)
        if (a.p[y].r1 <= 0 || a.p[y].r2 <= 0 || a.p[y].Q <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(probe_sum_kernel, dim3(S, 2), dim3(PB_THREADS), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small elementwise kernels.

__global__ void rowkron_kernel(int n, int r, int p, const double* __restrict__ Z, long ldz,
                               const double* __restrict__ X, long ldx, double* __restrict__ E) {
    const long total = (long)n * r * p;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % n);
        const long jc = e / n;
        const int j = int(jc % r), c = int(jc / r);
        E[e] = Z[i + ldz * j] * X[i + ldx * c];
    }
}

hipError_t rowkron(int n, int r, int p, const double* Z, long ldz, const double* X, long ldx,
                   double* E, hipStream_t s) {
    const long total = (long)n * r * p;
    if (total <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(rowkron_kernel, dim3(blocks), dim3(256), 0, s, n, r, p, Z, ldz, X, ldx, E);
    return hipGetLastError();
}

__global__ void rowcontract_kernel(int n, int r, int p, const double* __restrict__ Z, long ldz,
                                   const double* __restrict__ F, double* __restrict__ out,
                                   long ldo) {
    const long total = (long)n * p;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % n), c = int(e / n);
        double acc = 0.0;
        for (int j = 0; j < r; ++j) acc += Z[i + ldz * j] * F[i + (long)n * (j + (long)r * c)];
        out[i + ldo * c] = acc;
    }
}

hipError_t rowcontract(int n, int r, int p, const double* Z, long ldz, const double* F,
                       double* out, long ldo, hipStream_t s) {
    const long total = (long)n * p;
    if (total <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(rowcontract_kernel, dim3(blocks), dim3(256), 0, s, n, r, p, Z, ldz, F, out,
                       ldo);
    return hipGetLastError();
}

__global__ void rowkron_multi_kernel(int n, RowJobs jobs) {
    const RowJob& J = jobs.job[blockIdx.y];
    const long total = (long)n * J.r * J.p;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % n);
        const long jc = e / n;
        const int j = int(jc % J.r), c = int(jc / J.r);
        J.out[e] = J.Z[i + J.ldz * j] * J.X[i + J.ldx * c];
    }
}

hipError_t rowkron_multi(int n, const RowJobs& jobs, hipStream_t s) {
    long most = 0;
    for (int t = 0; t < jobs.count; ++t) most = std::max(most, (long)n * jobs.job[t].r * jobs.job[t].p);
    if (jobs.count <= 0 || most <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((most + 255) / 256, 8192);
    hipLaunchKernelGGL(rowkron_multi_kernel, dim3(blocks, jobs.count), dim3(256), 0, s, n, jobs);
    return hipGetLastError();
}

__global__ void rowcontract_multi_kernel(int n, RowJobs jobs) {
    const RowJob& J = jobs.job[blockIdx.y];
    const long total = (long)n * J.p;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % n), c = int(e / n);
        double acc = 0.0;
        for (int j = 0; j < J.r; ++j)
            acc += J.Z[i + J.ldz * j] * J.X[i + (long)n * (j + (long)J.r * c)];
        J.out[i + J.ldo * c] = acc;
    }
}

hipError_t rowcontract_multi(int n, const RowJobs& jobs, hipStream_t s) {
    long most = 0;
    for (int t = 0; t < jobs.count; ++t) most = std::max(most, (long)n * jobs.job[t].p);
    if (jobs.count <= 0 || most <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((most + 255) / 256, 8192);
    hipLaunchKernelGGL(rowcontract_multi_kernel, dim3(blocks, jobs.count), dim3(256), 0, s, n,
                       jobs);
    return hipGetLastError();
}

__global__ void permute_kernel(int r0, int r1, int r2, int mode, const double* __restrict__ src,
                               long sstride, double* __restrict__ dst, long dstride) {
    const long total = (long)r0 * r1 * r2;
    const double* S = src + blockIdx.y * sstride;
    double* D = dst + blockIdx.y * dstride;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % r0);
        const long t = e / r0;
        const int j = int(t % r1), kk = int(t / r1);
        long o;
        if (mode == 0) o = e;
        else if (mode == 1) o = j + (long)r1 * (i + (long)r0 * kk);
        else o = kk + (long)r2 * (i + (long)r0 * j);
        D[o] = S[e];
    }
}

// modes 1 and 2 of one core in one launch (grid.y picks the mode)
__global__ void permute12_kernel(int r0, int r1, int r2, const double* __restrict__ src,
                                 double* __restrict__ dst1, double* __restrict__ dst2) {
    const long total = (long)r0 * r1 * r2;
    const bool m1 = blockIdx.y == 0;
    double* D = m1 ? dst1 : dst2;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % r0);
        const long t = e / r0;
        const int j = int(t % r1), kk = int(t / r1);
        const long o = m1 ? j + (long)r1 * (i + (long)r0 * kk) : kk + (long)r2 * (i + (long)r0 * j);
        D[o] = src[e];
    }
}

hipError_t permute_core12(int r0, int r1, int r2, const double* src, double* dst1, double* dst2,
                          hipStream_t s) {
    const long total = (long)r0 * r1 * r2;
    if (total <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(permute12_kernel, dim3(blocks, 2), dim3(256), 0, s, r0, r1, r2, src, dst1,
                       dst2);
    return hipGetLastError();
}

hipError_t permute_core(int r0, int r1, int r2, int mode, int batch, const double* src,
                        long sstride, double* dst, long dstride, hipStream_t s) {
    const long total = (long)r0 * r1 * r2;
    if (total <= 0 || batch <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(permute_kernel, dim3(blocks, batch), dim3(256), 0, s, r0, r1, r2, mode, src,
                       sstride, dst, dstride);
    return hipGetLastError();
}

__global__ void axpby_kernel(long n, double a, const double* __restrict__ x, double b,
                             double* __restrict__ y) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        y[i] = a * x[i] + (b != 0.0 ? b * y[i] : 0.0);
}

hipError_t axpby(long n, double a, const double* x, double b, double* y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(axpby_kernel, dim3(blocks), dim3(256), 0, s, n, a, x, b, y);
    return hipGetLastError();
}

// x . y in one launch: each block writes its partial sum, and the block that
// counts in last (device-scope fences around the counter) adds the partial
// sums in block order, so the result does not depend on which block that is;
// it then resets the counter for the next call.
__global__ __launch_bounds__(256) void dot_kernel(long n, const double* __restrict__ x,
                                                  const double* __restrict__ y, double* part,
                                                  unsigned* count, double* out) {
    __shared__ double red[4];
    __shared__ int last;
    double acc = 0.0;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        acc += x[i] * y[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(&part[blockIdx.x], red[0] + red[1] + red[2] + red[3], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        last = atomicAdd(count, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double s = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += 256)   // gridDim.x <= 256: one each
        s += __hip_atomic_load(&part[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s = wave_sum(s);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = red[0] + red[1] + red[2] + red[3];
        atomicExch(count, 0u);
    }
}

hipError_t dot_long(long n, const double* x, const double* y, double* part, unsigned* count,
                    double* out, hipStream_t s) {
    const int parts = (int)std::min<long>(256, std::max<long>(1, (n + 4095) / 4096));
    hipLaunchKernelGGL(dot_kernel, dim3(parts), dim3(256), 0, s, n, x, y, part, count, out);
    return hipGetLastError();
}

__global__ void scale_cols_kernel(int n, int m, double* X, long ldx, const double* scale,
                                  int divide) {
    const long total = (long)n * m;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % n), c = int(e / n);
        const double f = scale[c];
        X[i + ldx * c] = divide ? (f != 0.0 ? X[i + ldx * c] / f : 0.0) : X[i + ldx * c] * f;
    }
}

hipError_t scale_cols(int n, int m, double* X, long ldx, const double* scale, int divide,
                      hipStream_t s) {
    const long total = (long)n * m;
    if (total <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_cols_kernel, dim3(blocks), dim3(256), 0, s, n, m, X, ldx, scale,
                       divide);
    return hipGetLastError();
}

__device__ void col_norm(int n, const double* __restrict__ x, double* out, double* red) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += x[i] * x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(red[0]);
}

// Column norms of up to kMaxPanelJobs matrices in one launch (grid.y).
__global__ __launch_bounds__(256) void col_norms_multi_kernel(int n, NormJobs jobs) {
    __shared__ double red[256];
    const NormJob& jb = jobs.job[blockIdx.y];
    if ((int)blockIdx.x >= jb.m) return;
    col_norm(n, jb.X + (long)blockIdx.x * n, jb.out + blockIdx.x, red);
}

hipError_t col_norms(int n, const NormJobs& jobs, hipStream_t s) {
    if (jobs.count <= 0) return hipSuccess;
    if (jobs.count > kMaxPanelJobs) return hipErrorInvalidValue;
    int mmax = 0;
    for (int t = 0; t < jobs.count; ++t) mmax = std::max(mmax, jobs.job[t].m);
    if (mmax <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_norms_multi_kernel, dim3(mmax, jobs.count), dim3(256), 0, s, n, jobs);
    return hipGetLastError();
}

__device__ inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void fill_random_multi_kernel(FillJobs jobs) {
    const FillJob& J = jobs.job[blockIdx.y];
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < J.n;
         i += (long)gridDim.x * blockDim.x) {
        const uint64_t h1 = splitmix64(((uint64_t)J.seed << 40) ^ (uint64_t)(2 * i));
        const uint64_t h2 = splitmix64(((uint64_t)J.seed << 40) ^ (uint64_t)(2 * i + 1));
        const double u1 = ((h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double u2 = ((h2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        J.x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

hipError_t fill_random_multi(const FillJobs& jobs, hipStream_t s) {
    long most = 0;
    for (int t = 0; t < jobs.count; ++t) most = std::max(most, jobs.job[t].n);
    if (jobs.count <= 0 || most <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((most + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_random_multi_kernel, dim3(blocks, jobs.count), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

// One workgroup per column t: U_l[:, t] /= ||U_l[:, t]|| for l = 0..2 and
// w[t] *= the product of the three norms.
__global__ void normalize_factors_kernel(int n, double* U0, double* U1, double* U2, long ld,
                                         double* w) {
    __shared__ double red[4];
    const int t = blockIdx.x, tid = threadIdx.x;
    double* U[3] = {U0 + (long)t * ld, U1 + (long)t * ld, U2 + (long)t * ld};
    double prod = 1.0;
    for (int l = 0; l < 3; ++l) {
        double s = 0.0;
        for (int i = tid; i < n; i += 256) s += U[l][i] * U[l][i];
        s = wave_sum(s);
        if ((tid & 63) == 0) red[tid >> 6] = s;
        __syncthreads();
        const double nrm = sqrt(red[0] + red[1] + red[2] + red[3]);
        __syncthreads();
        const double f = nrm > 0 ? 1.0 / nrm : 0.0;
        for (int i = tid; i < n; i += 256) U[l][i] *= f;
        prod *= nrm;
    }
    if (tid == 0) w[t] *= prod;
}

hipError_t normalize_factors(int n, int K, double* U0, double* U1, double* U2, long ld, double* w,
                             hipStream_t s) {
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(normalize_factors_kernel, dim3(K), dim3(256), 0, s, n, U0, U1, U2, ld, w);
    return hipGetLastError();
}

// d = 2 plans carry the third mode as one fixed eigenvector v: the design's
// mode-3 factor is v in every column, and the result's weights absorb the
// mode-3 factor's component along v.
__global__ void fill_columns_kernel(int n, int m, const double* __restrict__ v,
                                    double* __restrict__ out, long ld) {
    const long total = (long)n * m;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % n), j = int(e / n);
        out[i + ld * j] = v[i];
    }
}

hipError_t fill_columns(int n, int m, const double* v, double* out, long ld, hipStream_t s) {
    if (n <= 0 || m <= 0) return hipSuccess;
    const long total = (long)n * m;
    const int blocks = (int)std::min<long>((total + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_columns_kernel, dim3(blocks), dim3(256), 0, s, n, m, v, out, ld);
    return hipGetLastError();
}

// w[k] *= <U[:, k], v>, one workgroup of 256 per column.
__global__ void scale_by_dot_kernel(int n, const double* __restrict__ U, long ld,
                                    const double* __restrict__ v, double* __restrict__ w) {
    __shared__ double red[4];
    const int k = blockIdx.x, tid = threadIdx.x;
    const double* u = U + (long)k * ld;
    double acc = 0.0;
    for (int i = tid; i < n; i += 256) acc += u[i] * v[i];
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) w[k] *= (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t scale_by_dot(int n, int K, const double* U, long ld, const double* v, double* w,
                        hipStream_t s) {
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_by_dot_kernel, dim3(K), dim3(256), 0, s, n, U, ld, v, w);
    return hipGetLastError();
}

__global__ void copy2d_kernel(int rows, int cols, const double* __restrict__ src, long lds,
                              double* __restrict__ dst, long ldd) {
    const long total = (long)rows * cols;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % rows), j = int(e / rows);
        dst[i + ldd * j] = src ? src[i + lds * j] : 0.0;
    }
}

hipError_t copy2d(int rows, int cols, const double* src, long lds, double* dst, long ldd,
                  hipStream_t s) {
    const long total = (long)rows * cols;
    if (total <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(copy2d_kernel, dim3(blocks), dim3(256), 0, s, rows, cols, src, lds, dst,
                       ldd);
    return hipGetLastError();
}

__global__ void copy_multi_kernel(CopyJobs jobs) {
    const CopyJob& J = jobs.job[blockIdx.y];
    const long total = (long)J.rows * J.cols;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % J.rows), j = int(e / J.rows);
        J.dst[i + J.ldd * j] = J.src[i + J.lds * j];
    }
}

hipError_t copy_multi(const CopyJobs& jobs, hipStream_t s) {
    long most = 0;
    for (int t = 0; t < jobs.count; ++t)
        most = std::max(most, (long)jobs.job[t].rows * jobs.job[t].cols);
    if (jobs.count <= 0 || most <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((most + 255) / 256, 1024);
    hipLaunchKernelGGL(copy_multi_kernel, dim3(blocks, jobs.count), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

__global__ void sym_blocks_kernel(SymJobs jobs) {
    const SymJob& J = jobs.job[blockIdx.y];
    const long total = (long)J.k * J.k;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % J.k), j = int(e / J.k);
        int bi = 0, bj = 0;
        for (int t = 1; t < J.nb; ++t) {
            bi += i >= J.off[t];
            bj += j >= J.off[t];
        }
        // element (j, i) lies in a block above the diagonal: never written here
        if (bi > bj) J.M[i + (long)j * J.k] = J.M[j + (long)i * J.k];
    }
}

hipError_t sym_blocks(const SymJobs& jobs, hipStream_t s) {
    long most = 0;
    for (int t = 0; t < jobs.count; ++t) {
        if (jobs.job[t].nb < 1 || jobs.job[t].nb > kMaxSymBlocks) return hipErrorInvalidValue;
        most = std::max(most, (long)jobs.job[t].k * jobs.job[t].k);
    }
    if (jobs.count <= 0 || most <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((most + 255) / 256, 1024);
    hipLaunchKernelGGL(sym_blocks_kernel, dim3(blocks, jobs.count), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

__global__ void check_finite_kernel(long n, const double* __restrict__ x, int* flag) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) atomicOr(flag, 1);
}

hipError_t check_finite(long n, const double* x, int* flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(check_finite_kernel, dim3(blocks), dim3(256), 0, s, n, x, flag);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void cp_inner_kernel(int ra, int rb, const double* G0,
                                                       const double* G1, const double* G2,
                                                       const double* wa, const double* wb,
                                                       double* out) {
    __shared__ double red[256];
    double acc = 0.0;
    const long total = (long)ra * rb;
    for (long e = threadIdx.x; e < total; e += 256) {
        const int kk = int(e % ra), m = int(e / ra);
        acc += (wa ? wa[kk] : 1.0) * (wb ? wb[m] : 1.0) * G0[e] * G1[e] * G2[e];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t cp_inner_reduce(int ra, int rb, const double* G0, const double* G1, const double* G2,
                           const double* wa, const double* wb, double* out, hipStream_t s) {
    hipLaunchKernelGGL(cp_inner_kernel, dim3(1), dim3(256), 0, s, ra, rb, G0, G1, G2, wa, wb, out);
    return hipGetLastError();
}

// Block-wide sum of one value per thread (blockDim.x == 1024).
__device__ inline double block_sum_1024(double v, double* red) {
    const int tid = threadIdx.x;
    v = wave_sum(v);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    // every wavefront sums the 16 partials itself (no second barrier pair)
    const double r = wave_sum((tid & 63) < 16 ? red[tid & 63] : 0.0);
    __syncthreads();
    return r;
}

__global__ void transpose_kernel(int rows, int cols, const double* __restrict__ src, long lds,
                                 double* __restrict__ dst, long ldd) {
    const long total = (long)rows * cols;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int i = int(e % rows), j = int(e / rows);
        dst[j + ldd * i] = src[i + lds * j];
    }
}

hipError_t transpose(int rows, int cols, const double* src, long lds, double* dst, long ldd,
                     hipStream_t s) {
    const long total = (long)rows * cols;
    if (total <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(transpose_kernel, dim3(blocks), dim3(256), 0, s, rows, cols, src, lds, dst,
                       ldd);
    return hipGetLastError();
}

// Two-pass classical Gram-Schmidt inside a panel held in LDS: for column j,
// all dot products against the kept panel columns are formed in one sweep
// (one wavefront per column), then subtracted in one sweep.
__global__ __launch_bounds__(1024) void panel_mgs_kernel(int n, PanelJobs jobs, int passes) {
    extern __shared__ double P[];   // n x b
    __shared__ double red[32];
    __shared__ double dots[32];
    __shared__ int kp[32];
    const PanelJob& jb = jobs.job[blockIdx.x];
    double* Y = jb.Y;
    const double* norm0 = jb.norm0;
    const double drop = jb.drop;
    int* keep = jb.keep;
    const int b = jb.b;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // the panel into LDS, eight loads per thread in flight
    const long total = (long)n * b;
    for (long x0 = 0; x0 < total; x0 += 8 * 1024) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long x = x0 + tid + (long)u * 1024;
            v[u] = x < total ? Y[x] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long x = x0 + tid + (long)u * 1024;
            if (x < total) P[x] = v[u];
        }
    }
    __syncthreads();
    for (int j = 0; j < b; ++j) {
        double* y = P + (long)j * n;
        for (int pass = 0; pass < passes; ++pass) {
            if (j > 0) {
                for (int c = w; c < j; c += 16) {
                    double acc = 0.0;
                    if (kp[c]) {
                        const double* q = P + (long)c * n;
                        for (int i = lane; i < n; i += 64) acc += q[i] * y[i];
                    }
                    acc = wave_sum(acc);
                    if (lane == 0) dots[c] = acc;
                }
                __syncthreads();
                for (int i = tid; i < n; i += 1024) {
                    double v = y[i];
                    for (int c = 0; c < j; ++c) v -= dots[c] * P[(long)c * n + i];
                    y[i] = v;
                }
                __syncthreads();
            }
        }
        double s = 0.0;
        for (int i = tid; i < n; i += 1024) s += y[i] * y[i];
        const double nrm = sqrt(block_sum_1024(s, red));
        const bool ok = nrm > drop * (norm0 ? norm0[j] : 1.0) && nrm > 1e-300;
        const double f = ok ? 1.0 / nrm : 0.0;
        for (int i = tid; i < n; i += 1024) y[i] *= f;
        if (tid == 0) { kp[j] = ok ? 1 : 0; keep[j] = ok ? 1 : 0; }
        __syncthreads();
    }
    for (long x = tid; x < (long)n * b; x += 1024) Y[x] = P[x];
}

hipError_t panel_mgs(int n, const PanelJobs& jobs, int passes, hipStream_t s) {
    if (jobs.count <= 0) return hipSuccess;
    if (jobs.count > kMaxPanelJobs) return hipErrorInvalidValue;
    int bmax = 0;
    for (int i = 0; i < jobs.count; ++i) {
        if (jobs.job[i].b <= 0 || jobs.job[i].b > 32) return hipErrorInvalidValue;
        bmax = std::max(bmax, jobs.job[i].b);
    }
    if ((long)n * bmax * sizeof(double) > 144L * 1024) return hipErrorInvalidValue;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] {
        attr_err = hipFuncSetAttribute((const void*)panel_mgs_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    });
    if (attr_err != hipSuccess) return attr_err;
    hipLaunchKernelGGL(panel_mgs_kernel, dim3(jobs.count), dim3(1024), sizeof(double) * n * bmax, s,
                       n, jobs, passes);
    return hipGetLastError();
}

// Block projection update of a panel, P -= Y C (P n x b, Y n x j0, C j0 x b
// with leading dimension j0, b <= 16), for up to kMaxPanelJobs panels per
// launch (grid.y).  A workgroup covers 64 rows; its wavefront w handles the
// columns w, w + 4, ... of those rows, streaming the rows of Y (coalesced
// within the wavefront; the four wavefronts share them through the cache)
// against C held in LDS.
__global__ __launch_bounds__(256) void panel_update_kernel(int n, UpdateJobs jobs) {
    __shared__ double Cs[256 * 16];
    const UpdateJob& jb = jobs.job[blockIdx.y];
    const int j0 = jb.j0, b = jb.b;
    for (int x = threadIdx.x; x < j0 * b; x += 256) Cs[x] = jb.C[x];
    __syncthreads();
    const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + r;
    if (i >= n) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double* __restrict__ Y = jb.Y + i;
    // eight rows of C per step: eight independent loads of Y in flight
    int c = 0;
    for (; c + 8 <= j0; c += 8) {
        double y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u] = Y[(long)(c + u) * n];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = g + 4 * q;
                if (j < b) acc[q] += y[u] * Cs[c + u + j * j0];
            }
    }
    for (; c < j0; ++c) {
        const double y = Y[(long)c * n];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = g + 4 * q;
            if (j < b) acc[q] += y * Cs[c + j * j0];
        }
    }
    double* __restrict__ P = jb.P + i;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = g + 4 * q;
        if (j < b) P[(long)j * n] -= acc[q];
    }
}

hipError_t panel_update(int n, const UpdateJobs& jobs, hipStream_t s) {
    if (jobs.count <= 0) return hipSuccess;
    if (jobs.count > kMaxPanelJobs) return hipErrorInvalidValue;
    for (int t = 0; t < jobs.count; ++t)
        if (jobs.job[t].b < 1 || jobs.job[t].b > 16 || jobs.job[t].j0 < 1 || jobs.job[t].j0 > 256)
            return hipErrorInvalidValue;
    hipLaunchKernelGGL(panel_update_kernel, dim3((n + 63) / 64, jobs.count), dim3(256), 0, s, n,
                       jobs);
    return hipGetLastError();
}

// In-place compaction of the kept columns in one launch (grid.y: one job per
// matrix).  Every workgroup first turns keep[] into destinations (an
// exclusive prefix count, one wavefront, 64 flags per step by ballot +
// popcount; columns j < done count as kept) in LDS, then each thread moves
// its own row: columns in increasing order, column j to column pos[j] <= j.
// A row is only ever touched by its thread, and pos[j'] < j for every j' < j,
// so no source is overwritten before it is read.
__global__ __launch_bounds__(256) void compact_cols_kernel(int n, CompactJobs jobs) {
    __shared__ int pos[512];
    const CompactJob& jb = jobs.job[blockIdx.y];
    const int m = jb.m, done = jb.done;
    double* __restrict__ Y = jb.Y;
    const int tid = threadIdx.x;
    if (tid < 64) {
        int carry = 0;
        for (int base = 0; base < m; base += 64) {
            const int j = base + tid;
            const bool k = j < m && (j < done || jb.keep[j] != 0);
            const unsigned long long mask = __ballot(k);
            const int before = __popcll(mask & ((1ull << tid) - 1ull));
            if (j < m) pos[j] = k ? carry + before : -1;
            carry += __popcll(mask);
        }
        if (tid == 0 && blockIdx.x == 0) *jb.count = carry;
    }
    __syncthreads();
    const int i = blockIdx.x * 256 + tid;
    if (i >= n) return;
    for (int j = 0; j < m; ++j) {
        const int p = pos[j];
        if (p >= 0 && p != j) Y[i + (long)p * n] = Y[i + (long)j * n];
    }
}

hipError_t compact_cols(int n, const CompactJobs& jobs, hipStream_t s) {
    if (jobs.count <= 0) return hipSuccess;
    if (jobs.count > kMaxPanelJobs) return hipErrorInvalidValue;
    for (int i = 0; i < jobs.count; ++i)
        if (jobs.job[i].m < 0 || jobs.job[i].m > 512) return hipErrorInvalidValue;
    hipLaunchKernelGGL(compact_cols_kernel, dim3((n + 255) / 256, jobs.count), dim3(256), 0, s, n,
                       jobs);
    return hipGetLastError();
}

// One 16x16x4 product of fixed matrices, written out with the accumulator
// layout assumed by the GEMM (used by a self-test).
__global__ void mfma_probe_kernel(double* out) {
    const int lane = threadIdx.x;
    const int i = lane & 15, k = lane >> 4;
    const double a = 1.0 + i + 16.0 * k;           // A[i][k]
    const double b = 1.0 + 0.5 * k - 0.25 * i;     // B[k][j], j = lane & 15
    dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    for (int v = 0; v < 4; ++v) {
        const int row = (lane >> 4) + 4 * v, col = lane & 15;
        out[row * 16 + col] = acc[v];
    }
}

// The same product on the FP32 matrix core (v_mfma_f32_16x16x4f32); out[256..511]
// receives the accumulator with the row mapping used by the FP32 GEMM.
__global__ void mfma_probe_f32_kernel(double* out) {
    const int lane = threadIdx.x;
    const int i = lane & 15, k = lane >> 4;
    const float a = 1.0f + i + 16.0f * k;
    const float b = 1.0f + 0.5f * k - 0.25f * i;
    flt4 acc = flt4{0.0f, 0.0f, 0.0f, 0.0f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    for (int v = 0; v < 4; ++v) {
        const int row = F32_ROW(lane, v), col = lane & 15;
        out[256 + row * 16 + col] = acc[v];
    }
}

hipError_t mfma_probe(double* out, hipStream_t s) {
    hipLaunchKernelGGL(mfma_probe_f32_kernel, dim3(1), dim3(64), 0, s, out);
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
}

}  // namespace fc
