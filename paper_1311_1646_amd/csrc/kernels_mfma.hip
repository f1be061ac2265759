// Grouped block GEMM on the CDNA4 matrix cores (gfx950).
//
// Same work lists as the FP64 FMA kernel (tiles / jobs / contributions with
// base-relative addressing).  A workgroup of four waves owns one 64x64 output
// tile; each wave owns a 32x32 quarter.  Every contribution of the job is
// streamed through LDS in K-chunks of 16 with the op() transposition applied
// while staging, zero-filled outside the block (ragged edges).
//   FP64 : v_mfma_f64_16x16x4f64, 2x2 per wave, FP64 accumulate
//          (16x16 result: lane l, register r holds row (l/16) + 4r, column l%16).
//   FP32 : v_mfma_f32_32x32x2f32, FP32 accumulate (32x32 result: lane l,
//          register r holds row 8(r/4) + 4(l/32) + r%4, column l%32).
//   BF16X3 : each FP32 operand split x = hi + lo (bfloat16), three
//            v_mfma_f32_32x32x16_bf16 products hi*hi + hi*lo + lo*hi, FP32
//            accumulate (about 2^-16 relative per product).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "kernels_mfma.hpp"

namespace dmrg {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64, TN = 64, TK = 16, NTH = 256;

template <class T>
__device__ __forceinline__ const T* cptr(const Bases& b, int base, long off, int bz) {
  return reinterpret_cast<const T*>(b.p[base]) + off + long(bz) * b.stride[base];
}
template <class T>
__device__ __forceinline__ T* mptr(const Bases& b, int base, long off, int bz) {
  return reinterpret_cast<T*>(b.p[base]) + off + long(bz) * b.stride[base];
}

// Stage op(A) (TM x TK) and op(B) (TK x TN) of one K-chunk into LDS, both
// stored row-per-output-index: As[i][k], Bs[j][k].
template <class T>
__device__ __forceinline__ void stage(T (*As)[TK + 1], T (*Bs)[TK + 1], const GContrib& c, const T* A,
                                      const T* B, int m, int n, int row0, int col0, int k0, int tid) {
  const bool ta = c.flags & GC_TRANS_A, tb = c.flags & GC_TRANS_B, aid = c.flags & GC_A_IDENTITY;
  const T alpha = T(c.alpha);
#pragma unroll
  for (int q = 0; q < (TM * TK) / NTH; ++q) {
    const int e = tid + q * NTH;
    int i, k;
    if (ta) { k = e / TM; i = e % TM; } else { i = e / TK; k = e % TK; }
    const int gi = row0 + i, gk = k0 + k;
    T v = T(0);
    if (gi < m && gk < c.k) {
      if (aid) v = gi == gk ? T(1) : T(0);
      else v = ta ? A[long(gk) * c.lda + gi] : A[long(gi) * c.lda + gk];
    }
    As[i][k] = v * alpha;
  }
#pragma unroll
  for (int q = 0; q < (TN * TK) / NTH; ++q) {
    const int e = tid + q * NTH;
    int j, k;
    if (tb) { j = e / TK; k = e % TK; } else { k = e / TN; j = e % TN; }
    const int gj = col0 + j, gk = k0 + k;
    T v = T(0);
    if (gk < c.k && gj < n) v = tb ? B[long(gj) * c.ldb + gk] : B[long(gk) * c.ldb + gj];
    Bs[j][k] = v;
  }
}

__device__ __forceinline__ void split_bf16(const float* x, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const __bf16 h = static_cast<__bf16>(x[t]);
    hi[t] = h;
    lo[t] = static_cast<__bf16>(x[t] - static_cast<float>(h));
  }
}

template <class TOut>
__device__ __forceinline__ void store_out(TOut* C, const GJob& J, int r, int c, float v) {
  if (r < J.m && c < J.n) {
    TOut* p = C + long(r) * J.ldc + c;
    *p = (J.flags & GJ_ACCUMULATE) ? TOut(*p + TOut(v)) : TOut(v);
  }
}

// MODE 1: FP32 MFMA, MODE 2: BF16x3 MFMA (FP32 data in memory)
template <int MODE, class TOut>
__global__ __launch_bounds__(NTH) void ggemm_f32_kernel(const GTile* __restrict__ tiles, const GJob* __restrict__ jobs,
                                                        const GContrib* __restrict__ con, Bases bs, Bases bout) {
  __shared__ float As[TM][TK + 1];
  __shared__ float Bs[TN][TK + 1];
  const GTile t = tiles[blockIdx.x];
  const GJob J = jobs[t.job];
  const int bz = blockIdx.y;
  const int row0 = t.tm * TM, col0 = t.tn * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  floatx16 acc = {0};
  for (int ci = J.c0; ci < J.c1; ++ci) {
    const GContrib c = con[ci];
    const float* A = (c.flags & GC_A_IDENTITY) ? nullptr : cptr<float>(bs, c.baseA, c.offA, bz);
    const float* B = cptr<float>(bs, c.baseB, c.offB, bz);
    for (int k0 = 0; k0 < c.k; k0 += TK) {
      stage<float>(As, Bs, c, A, B, J.m, J.n, row0, col0, k0, tid);
      __syncthreads();
      if (MODE == 1) {
#pragma unroll
        for (int s = 0; s < TK / 2; ++s) {
          const int k = 2 * s + (lane >> 5);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[wm + (lane & 31)][k], Bs[wn + (lane & 31)][k], acc, 0, 0, 0);
        }
      } else {
        float av[8], bv[8];
        const int kb = 8 * (lane >> 5);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          av[q] = As[wm + (lane & 31)][kb + q];
          bv[q] = Bs[wn + (lane & 31)][kb + q];
        }
        bf16x8 ah, al, bh, bl;
        split_bf16(av, ah, al);
        split_bf16(bv, bh, bl);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
      }
      __syncthreads();
    }
  }
  TOut* C = mptr<TOut>(bout, J.baseC, J.offC, bz);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    store_out<TOut>(C, J, row0 + wm + i, col0 + wn + (lane & 31), acc[r]);
  }
}

__global__ __launch_bounds__(NTH) void ggemm_f64_mfma_kernel(const GTile* __restrict__ tiles,
                                                             const GJob* __restrict__ jobs,
                                                             const GContrib* __restrict__ con, Bases bs) {
  __shared__ double As[TM][TK + 1];
  __shared__ double Bs[TN][TK + 1];
  const GTile t = tiles[blockIdx.x];
  const GJob J = jobs[t.job];
  const int bz = blockIdx.y;
  const int row0 = t.tm * TM, col0 = t.tn * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  doublex4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = doublex4{0, 0, 0, 0};
  for (int ci = J.c0; ci < J.c1; ++ci) {
    const GContrib c = con[ci];
    const double* A = (c.flags & GC_A_IDENTITY) ? nullptr : cptr<double>(bs, c.baseA, c.offA, bz);
    const double* B = cptr<double>(bs, c.baseB, c.offB, bz);
    for (int k0 = 0; k0 < c.k; k0 += TK) {
      stage<double>(As, Bs, c, A, B, J.m, J.n, row0, col0, k0, tid);
      __syncthreads();
#pragma unroll
      for (int s = 0; s < TK / 4; ++s) {
        const int k = 4 * s + (lane >> 4);
        double av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = As[wm + 16 * a + (lane & 15)][k];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Bs[wn + 16 * b + (lane & 15)][k];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  double* C = mptr<double>(bs, J.baseC, J.offC, bz);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + wm + 16 * a + (lane >> 4) + 4 * r;
        const int j = col0 + wn + 16 * b + (lane & 15);
        if (i < J.m && j < J.n) {
          double* p = C + long(i) * J.ldc + j;
          *p = (J.flags & GJ_ACCUMULATE) ? *p + acc[a][b][r] : acc[a][b][r];
        }
      }
}

__global__ void lincomb_f32_kernel(const LCTarget* __restrict__ tg, const LCSource* __restrict__ src, Bases bs) {
  const LCTarget t = tg[blockIdx.y];
  const int bz = blockIdx.z;
  float* out = mptr<float>(bs, t.base, t.off, bz);
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < t.size; e += long(gridDim.x) * blockDim.x) {
    float s = 0.f;
    for (int j = t.s0; j < t.s1; ++j) s = fmaf(float(src[j].c), cptr<float>(bs, src[j].base, src[j].off, bz)[e], s);
    out[e] = t.accumulate ? out[e] + s : s;
  }
}

__global__ void diag_add_f32_kernel(const DiagAdd* __restrict__ d, Bases bs) {
  const DiagAdd x = d[blockIdx.x];
  float* o = mptr<float>(bs, x.base, x.off, blockIdx.y);
  for (int i = threadIdx.x; i < x.dim; i += blockDim.x) o[long(i) * (x.dim + 1)] += float(x.c);
}

__global__ void convert_f64_f32_kernel(const double* __restrict__ in, float* __restrict__ out, long n) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x)
    out[e] = float(in[e]);
}

}  // namespace

void launch_grouped_gemm(int prec, bool out_f64, const GTile* tiles, int ntiles, const GJob* jobs, const GContrib* con,
                         const Bases& b, const Bases& bout, int batch, hipStream_t s) {
  if (ntiles <= 0 || batch <= 0) return;
  const dim3 grid(ntiles, batch), block(NTH);
  if (prec == 0) {
    hipLaunchKernelGGL(ggemm_f64_mfma_kernel, grid, block, 0, s, tiles, jobs, con, b);
  } else if (prec == 1) {
    if (out_f64) hipLaunchKernelGGL((ggemm_f32_kernel<1, double>), grid, block, 0, s, tiles, jobs, con, b, bout);
    else hipLaunchKernelGGL((ggemm_f32_kernel<1, float>), grid, block, 0, s, tiles, jobs, con, b, bout);
  } else {
    if (out_f64) hipLaunchKernelGGL((ggemm_f32_kernel<2, double>), grid, block, 0, s, tiles, jobs, con, b, bout);
    else hipLaunchKernelGGL((ggemm_f32_kernel<2, float>), grid, block, 0, s, tiles, jobs, con, b, bout);
  }
}

void launch_lincomb_f32(const LCTarget* t, int ntargets, const LCSource* src, long max_size, const Bases& b, int batch,
                        hipStream_t s) {
  if (ntargets <= 0 || max_size <= 0 || batch <= 0) return;
  long blocks = (max_size + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  for (int t0 = 0; t0 < ntargets; t0 += 65535) {
    const int nt = ntargets - t0 < 65535 ? ntargets - t0 : 65535;
    hipLaunchKernelGGL(lincomb_f32_kernel, dim3(unsigned(blocks), nt, batch), dim3(256), 0, s, t + t0, src, b);
  }
}

void launch_diag_add_f32(const DiagAdd* d, int n, const Bases& b, int batch, hipStream_t s) {
  if (n <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(diag_add_f32_kernel, dim3(n, batch), dim3(256), 0, s, d, b);
}

void launch_convert_f64_f32(const double* in, float* out, long n, hipStream_t s) {
  if (n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(convert_f64_f32_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, in, out, n);
}

}  // namespace dmrg
