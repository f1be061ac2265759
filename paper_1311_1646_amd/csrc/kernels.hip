// FP64 device kernels of the block-sparse contractions.
#include "kernels.hpp"

namespace dmrg {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

// 64x64 output tile, 256 threads, 4x4 outputs per thread; every contribution
// of the job is streamed through LDS in K-chunks of 16.
__global__ __launch_bounds__(NT) void grouped_gemm_f64_kernel(const GTile* __restrict__ tiles,
                                                                const GJob* __restrict__ jobs,
                                                                const GContrib* __restrict__ con,
                                                                long sA, long sB, long sC) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const GTile t = tiles[blockIdx.x];
  const GJob J = jobs[t.job];
  const int bz = blockIdx.y;
  const int row0 = t.tm * BM, col0 = t.tn * BN;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int ci = J.c0; ci < J.c1; ++ci) {
    const GContrib c = con[ci];
    const double* A = static_cast<const double*>(c.A);
    const double* B = static_cast<const double*>(c.B);
    if (c.flags & GC_A_BATCHED) A += bz * sA;
    if (c.flags & GC_B_BATCHED) B += bz * sB;
    if (c.flags & GC_B_BATCHED_ALT) B += bz * sA;
    const bool ta = c.flags & GC_TRANS_A, tb = c.flags & GC_TRANS_B, aid = c.flags & GC_A_IDENTITY;
    for (int k0 = 0; k0 < c.k; k0 += BK) {
      for (int e = tid; e < BM * BK; e += NT) {
        int r, kk;
        if (ta) { kk = e / BM; r = e % BM; } else { r = e / BK; kk = e % BK; }
        const int gr = row0 + r, gk = k0 + kk;
        double v = 0.0;
        if (gr < J.m && gk < c.k) {
          if (aid) v = (gr == gk) ? 1.0 : 0.0;
          else v = ta ? A[long(gk) * c.lda + gr] : A[long(gr) * c.lda + gk];
        }
        As[kk][r] = v * c.alpha;
      }
      for (int e = tid; e < BK * BN; e += NT) {
        int kk, cc;
        if (tb) { cc = e / BK; kk = e % BK; } else { kk = e / BN; cc = e % BN; }
        const int gk = k0 + kk, gc = col0 + cc;
        double v = 0.0;
        if (gk < c.k && gc < J.n) v = tb ? B[long(gc) * c.ldb + gk] : B[long(gk) * c.ldb + gc];
        Bs[kk][cc] = v;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
      }
      __syncthreads();
    }
  }
  double* C = static_cast<double*>(J.C);
  if (J.flags & GJ_C_BATCHED) C += bz * sC;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = row0 + ty * 4 + i;
    if (r >= J.m) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cc = col0 + tx * 4 + j;
      if (cc >= J.n) continue;
      double* p = C + long(r) * J.ldc + cc;
      *p = (J.flags & GJ_ACCUMULATE) ? *p + acc[i][j] : acc[i][j];
    }
  }
}

__global__ void lincomb_f64_kernel(const LCTarget* __restrict__ tg, const LCSource* __restrict__ src,
                                   long stride) {
  const LCTarget t = tg[blockIdx.y];
  const long off = long(blockIdx.z) * stride;
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < t.size; e += long(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int j = t.s0; j < t.s1; ++j) s = fma(src[j].c, src[j].src[off + e], s);
    double* o = t.out + off + e;
    *o = t.accumulate ? *o + s : s;
  }
}

__global__ void diag_add_f64_kernel(const DiagAdd* __restrict__ d) {
  const DiagAdd x = d[blockIdx.x];
  for (int i = threadIdx.x; i < x.dim; i += blockDim.x) x.out[long(i) * (x.dim + 1)] += x.c;
}

__global__ void fill_f64_kernel(double* p, long n, double v) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) p[e] = v;
}

__global__ void diag_jobs_f64_kernel(const DiagJob* __restrict__ jobs, const DiagTerm* __restrict__ t) {
  const DiagJob J = jobs[blockIdx.x];
  const int n = J.rows * J.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int l = e / J.cols, r = e % J.cols;
    double s = 0.0;
    for (int k = J.t0; k < J.t1; ++k) {
      const double a = t[k].X ? t[k].X[long(l) * (J.rows + 1)] : 1.0;
      const double b = t[k].Z ? t[k].Z[long(r) * (J.cols + 1)] : 1.0;
      s = fma(t[k].alpha * a, b, s);
    }
    J.out[e] = s;
  }
}

}  // namespace

void launch_grouped_gemm_f64(const GTile* tiles, int ntiles, const GJob* jobs, const GContrib* con,
                             int batch, long sA, long sB, long sC, hipStream_t s) {
  if (ntiles <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(grouped_gemm_f64_kernel, dim3(ntiles, batch), dim3(NT), 0, s, tiles, jobs, con, sA, sB, sC);
}

void launch_lincomb_f64(const LCTarget* t, int ntargets, const LCSource* src, long max_size, int batch,
                        long stride, hipStream_t s) {
  if (ntargets <= 0 || max_size <= 0) return;
  long blocks = (max_size + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  for (int t0 = 0; t0 < ntargets; t0 += 65535) {
    const int nt = ntargets - t0 < 65535 ? ntargets - t0 : 65535;
    hipLaunchKernelGGL(lincomb_f64_kernel, dim3(unsigned(blocks), nt, batch), dim3(256), 0, s, t + t0, src, stride);
  }
}

void launch_diag_add_f64(const DiagAdd* d, int n, int, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(diag_add_f64_kernel, dim3(n), dim3(256), 0, s, d);
}

void launch_fill_f64(double* p, long n, double v, hipStream_t s) {
  if (n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, n, v);
}

void launch_diag_jobs_f64(const DiagJob* j, int n, const DiagTerm* t, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(diag_jobs_f64_kernel, dim3(n), dim3(256), 0, s, j, t);
}

}  // namespace dmrg
