// FP64 device kernels: grouped block GEMM, operator linear combinations,
// diagonal of the effective Hamiltonian, dense vector kernels of the Davidson
// sweeps and the small generalized eigensolver.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "kernels.hpp"

namespace dmrg {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

__device__ __forceinline__ double* bptr(const Bases& b, int base, long off, int bz) {
  return b.p[base] + off + long(bz) * b.stride[base];
}

// 64x64 output tile, 256 threads, 4x4 outputs per thread; every contribution
// of the job is streamed through LDS in K-chunks of 16.
__global__ __launch_bounds__(NT) void grouped_gemm_f64_kernel(const GTile* __restrict__ tiles,
                                                                const GJob* __restrict__ jobs,
                                                                const GContrib* __restrict__ con,
                                                                const int* __restrict__ gather, Bases bs) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const GTile t = tiles[blockIdx.x];
  const GJob J = jobs[t.job];
  const int bz = blockIdx.y;
  const int row0 = t.tm * BM, col0 = t.tn * BN;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const bool ga = J.flags & GJ_GATHER_A, gb = J.flags & GJ_GATHER_B;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int ci = J.c0; ci < J.c1; ++ci) {
    const GContrib c = con[ci];
    const bool ta = c.flags & GC_TRANS_A, tb = c.flags & GC_TRANS_B, aid = c.flags & GC_A_IDENTITY;
    const double* A = aid ? nullptr : bptr(bs, c.baseA, c.offA, bz);
    const double* B = bptr(bs, c.baseB, c.offB, bz);
    for (int k0 = 0; k0 < c.k; k0 += BK) {
      for (int e = tid; e < BM * BK; e += NT) {
        int r, kk;
        if (ta) { kk = e / BM; r = e % BM; } else { r = e / BK; kk = e % BK; }
        const int gr = row0 + r, gk = k0 + kk;
        double v = 0.0;
        if (gr < J.m && gk < c.k) {
          if (aid) v = (gr == gk) ? 1.0 : 0.0;
          else if (ga) v = A[long(gather[J.pad + gr]) + gk];
          else v = ta ? A[long(gk) * c.lda + gr] : A[long(gr) * c.lda + gk];
        }
        As[kk][r] = v * c.alpha;
      }
      for (int e = tid; e < BK * BN; e += NT) {
        int kk, cc;
        if (tb) { cc = e / BK; kk = e % BK; } else { kk = e / BN; cc = e % BN; }
        const int gk = k0 + kk, gc = col0 + cc;
        double v = 0.0;
        if (gk < c.k && gc < J.n)
          v = gb ? B[long(gather[J.pad + gc]) + gk] : (tb ? B[long(gc) * c.ldb + gk] : B[long(gk) * c.ldb + gc]);
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
  double* C = bptr(bs, J.baseC, J.offC, bz);
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

__global__ void lincomb_f64_kernel(const LCTarget* __restrict__ tg, const LCSource* __restrict__ src, Bases bs) {
  const LCTarget t = tg[blockIdx.y];
  const int bz = blockIdx.z;
  double* out = bptr(bs, t.base, t.off, bz);
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < t.size; e += long(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int j = t.s0; j < t.s1; ++j) s = fma(src[j].c, bptr(bs, src[j].base, src[j].off, bz)[e], s);
    out[e] = t.accumulate ? out[e] + s : s;
  }
}

__global__ void diag_add_f64_kernel(const DiagAdd* __restrict__ d, Bases bs, const Bases* __restrict__ ib) {
  const DiagAdd x = d[blockIdx.x];
  double* o = bptr(ib ? ib[x.inst] : bs, x.base, x.off, blockIdx.y);
  for (int i = threadIdx.x; i < x.dim; i += blockDim.x) o[long(i) * (x.dim + 1)] += x.c;
}

__global__ void fill_f64_kernel(double* p, long n, double v) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) p[e] = v;
}

__global__ void add_f64_kernel(const double* __restrict__ x, double* __restrict__ y, long n) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) y[e] += x[e];
}

__global__ void zero_f32_kernel(float* p, long n) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) p[e] = 0.0f;
}

__global__ void diag_jobs_f64_kernel(const DiagJob* __restrict__ jobs, const DiagTerm* __restrict__ t, Bases bs) {
  const DiagJob J = jobs[blockIdx.x];
  const int n = J.rows * J.cols;
  double* out = bptr(bs, J.base, J.off, 0);
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int l = e / J.cols, r = e % J.cols;
    double s = 0.0;
    for (int k = J.t0; k < J.t1; ++k) {
      const double a = t[k].offX >= 0 ? bptr(bs, t[k].baseX, t[k].offX, 0)[long(l) * (J.rows + 1)] : 1.0;
      const double b = t[k].offZ >= 0 ? bptr(bs, t[k].baseZ, t[k].offZ, 0)[long(r) * (J.cols + 1)] : 1.0;
      s = fma(t[k].alpha * a, b, s);
    }
    out[e] = s;
  }
}

// ---- dense vector kernels

constexpr int GRAM_SUB = 32;
// Elements per partial sum of the Gram products: about 512 workgroups per
// product (two per compute unit), chunks of 256 to 4096 elements in steps of
// GRAM_SUB.  A fixed 4096 left vectors of 10^4-10^5 elements (a site at
// M = 100-300) with a few dozen workgroups, each looping 128 times.
long gram_chunk(long n) {
  long c = (n + 511) / 512;
  c = (c + GRAM_SUB - 1) / GRAM_SUB * GRAM_SUB;
  return c < 256 ? 256 : (c > 4096 ? 4096 : c);
}

__global__ __launch_bounds__(256) void gram_part_kernel(const double* __restrict__ A, long lda, int na,
                                                        const double* __restrict__ B, long ldb, int nb, long n,
                                                        long chunk, double* __restrict__ part) {
  __shared__ double As[64][GRAM_SUB + 1];
  __shared__ double Bs[64][GRAM_SUB + 1];
  const long e0 = long(blockIdx.x) * chunk;
  const long e1 = e0 + chunk < n ? e0 + chunk : n;
  const int tid = threadIdx.x;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (long s0 = e0; s0 < e1; s0 += GRAM_SUB) {
    for (int x = tid; x < 64 * GRAM_SUB; x += 256) {
      const int r = x / GRAM_SUB, k = x % GRAM_SUB;
      const long e = s0 + k;
      As[r][k] = (r < na && e < e1) ? A[long(r) * lda + e] : 0.0;
      Bs[r][k] = (r < nb && e < e1) ? B[long(r) * ldb + e] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = tid + q * 256, m = o / 64, kk = o % 64;
      if (m < na && kk < nb) {
        double s = 0.0;
        for (int k = 0; k < GRAM_SUB; ++k) s = fma(As[m][k], Bs[kk][k], s);
        acc[q] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int o = tid + q * 256, m = o / 64, kk = o % 64;
    if (m < na && kk < nb) part[(long(blockIdx.x) * na + m) * nb + kk] = acc[q];
  }
}

__global__ void gram_reduce_kernel(const double* __restrict__ part, int nparts, int na, int nb, double* G, int ldg,
                                   double alpha, int accumulate) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= na * nb) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[long(p) * na * nb + o];
  const int m = o / nb, k = o % nb;
  double* g = G + long(m) * ldg + k;
  *g = accumulate ? *g + alpha * s : alpha * s;
}

__global__ void axpby_kernel(const double* a, const double* x, long ldx, const double* b, double* y, long ldy,
                             long n) {
  const int v = blockIdx.y;
  const double av = a ? a[v] : 1.0, bv = b ? b[v] : 0.0;
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) {
    const double xv = x ? x[long(v) * ldx + e] : 0.0;
    double* yy = y + long(v) * ldy + e;
    *yy = bv == 0.0 ? av * xv : av * xv + bv * *yy;
  }
}

__global__ void precond_kernel(const double* r, const double* d, const double* w, double* z, long n, double eps) {
  const int v = blockIdx.y;
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) {
    double den = d[e] - w[v];
    if (fabs(den) < eps) den = den < 0 ? -eps : eps;
    z[long(v) * n + e] = r[long(v) * n + e] / den;
  }
}

__global__ void rotate_kernel(const double* __restrict__ X, long ldx, int nin, const double* __restrict__ A, int lda,
                              int nout, double* __restrict__ Y, long ldy, long n) {
  // outputs in chunks of RC held in registers (constant indices only: a
  // private array indexed at run time would live in scratch memory); X is
  // re-read once per chunk, from cache
  constexpr int RC = 16;
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) {
    for (int v0 = 0; v0 < nout; v0 += RC) {
      double acc[RC];
#pragma unroll
      for (int j = 0; j < RC; ++j) acc[j] = 0.0;
      for (int u = 0; u < nin; ++u) {
        const double xv = X[long(u) * ldx + e];
#pragma unroll
        for (int j = 0; j < RC; ++j)
          if (v0 + j < nout) acc[j] = fma(xv, A[u + (v0 + j) * lda], acc[j]);
      }
#pragma unroll
      for (int j = 0; j < RC; ++j)
        if (v0 + j < nout) Y[long(v0 + j) * ldy + e] = acc[j];
    }
  }
}

__global__ void block_scale_kernel(const BlockScale* bs, const double* vec, double* data, long stride) {
  const BlockScale b = bs[blockIdx.x];
  double* d = data + long(blockIdx.y) * stride + b.off;
  const int n = b.rows * b.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = e / b.cols, c = e % b.cols;
    d[e] *= vec[b.vec_off + (b.by_rows ? r : c)];
  }
}

// ---- small symmetric (generalized) eigensolver, one workgroup

constexpr int GN = 64;

// Parallel cyclic Jacobi (round-robin pairing) on the leading m x m block of
// A, rotations accumulated into V (initialized by the caller).
__device__ void jacobi_lds(double (*A)[GN + 1], double (*V)[GN + 1], int m, double* cs, int* pr, double* red) {
  const int tid = threadIdx.x;
  const int mm = (m + 1) & ~1;  // even count; index m is a phantom when m is odd
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) {
      double off = 0.0, nrm = 0.0;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          const double v = A[i][j] * A[i][j];
          nrm += v;
          if (i != j) off += v;
        }
      red[0] = (off <= 1e-30 * nrm) ? 1.0 : 0.0;
    }
    __syncthreads();
    const bool done = red[0] != 0.0;
    __syncthreads();
    if (done) break;
    for (int round = 0; round < mm - 1; ++round) {
      if (tid < mm / 2) {
        const int a = tid == 0 ? 0 : 1 + (tid - 1 + round) % (mm - 1);
        const int b = 1 + (mm - 2 - tid + round) % (mm - 1);
        const int p = a < b ? a : b, q = a < b ? b : a;
        pr[2 * tid] = p;
        pr[2 * tid + 1] = q;
        double c = 1.0, s = 0.0;
        if (q < m && A[p][q] != 0.0) {
          const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
          const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
      }
      __syncthreads();
      for (int x = tid; x < m * (mm / 2); x += blockDim.x) {
        const int r = x / (mm / 2), k = x % (mm / 2);
        const int p = pr[2 * k], q = pr[2 * k + 1];
        if (q >= m) continue;
        const double c = cs[2 * k], s = cs[2 * k + 1];
        const double ap = A[r][p], aq = A[r][q];
        A[r][p] = c * ap - s * aq;
        A[r][q] = s * ap + c * aq;
        const double vp = V[r][p], vq = V[r][q];
        V[r][p] = c * vp - s * vq;
        V[r][q] = s * vp + c * vq;
      }
      __syncthreads();
      for (int x = tid; x < m * (mm / 2); x += blockDim.x) {
        const int col = x / (mm / 2), k = x % (mm / 2);
        const int p = pr[2 * k], q = pr[2 * k + 1];
        if (q >= m) continue;
        const double c = cs[2 * k], s = cs[2 * k + 1];
        const double ap = A[p][col], aq = A[q][col];
        A[p][col] = c * ap - s * aq;
        A[q][col] = s * ap + c * aq;
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void gep_kernel(const double* H, const double* S, int n, double thr, double* w,
                                                  double* X, int* rank) {
  __shared__ double A[GN][GN + 1];
  __shared__ double V[GN][GN + 1];
  __shared__ double Y[GN][GN + 1];
  __shared__ double cs[GN];
  __shared__ int pr[GN];
  __shared__ int keep[GN];
  __shared__ double ev[GN];
  __shared__ double red[2];
  __shared__ int nk;
  const int tid = threadIdx.x;
  for (int x = tid; x < n * n; x += blockDim.x) {
    const int i = x / n, j = x % n;
    A[i][j] = 0.5 * (S[i * n + j] + S[j * n + i]);
    V[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_lds(A, V, n, cs, pr, red);
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, A[i][i]);
    int c = 0;
    for (int i = 0; i < n; ++i)
      if (A[i][i] > thr * mx && A[i][i] > 0.0) keep[c++] = i;
    nk = c;
    for (int i = 0; i < n; ++i) ev[i] = A[i][i];
  }
  __syncthreads();
  const int r = nk;
  for (int x = tid; x < n * r; x += blockDim.x) {
    const int i = x / r, k = x % r;
    Y[i][k] = V[i][keep[k]] / sqrt(ev[keep[k]]);
  }
  __syncthreads();
  for (int x = tid; x < n * r; x += blockDim.x) {
    const int i = x / r, k = x % r;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += 0.5 * (H[i * n + j] + H[j * n + i]) * Y[j][k];
    V[i][k] = s;
  }
  __syncthreads();
  for (int x = tid; x < r * r; x += blockDim.x) {
    const int k = x / r, l = x % r;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += Y[j][k] * V[j][l];
    A[k][l] = s;
  }
  __syncthreads();
  for (int x = tid; x < r * r; x += blockDim.x) {
    const int k = x / r, l = x % r;
    V[k][l] = k == l ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_lds(A, V, r, cs, pr, red);
  if (tid < r) {
    const double me = A[tid][tid];
    int pos = 0;
    for (int j = 0; j < r; ++j) {
      const double o = A[j][j];
      if (o < me || (o == me && j < tid)) ++pos;
    }
    keep[pos] = tid;
  }
  __syncthreads();
  for (int x = tid; x < n * n; x += blockDim.x) {
    const int i = x % n, k = x / n;  // column-major X
    double s = 0.0;
    if (k < r) {
      const int src = keep[k];
      for (int j = 0; j < r; ++j) s += Y[i][j] * V[j][src];
    }
    X[i + long(k) * n] = s;
  }
  if (tid < n) w[tid] = tid < r ? A[keep[tid]][keep[tid]] : DBL_MAX;
  if (tid == 0) *rank = r;
}

}  // namespace

void launch_grouped_gemm_f64(const GTile* tiles, int ntiles, const GJob* jobs, const GContrib* con,
                             const int* gather, const Bases& b, int batch, hipStream_t s) {
  if (ntiles <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(grouped_gemm_f64_kernel, dim3(ntiles, batch), dim3(NT), 0, s, tiles, jobs, con, gather, b);
}

// Each thread owns lc_elems<T>() elements a block width apart and reads
// kLCAhead sources for all of them before applying the coefficients, so a
// wave keeps several loads in flight instead of one.  Every element still
// sums its sources in list order.
template <class T>
__host__ __device__ constexpr int lc_elems() { return sizeof(T) == 8 ? 2 : 4; }
constexpr int kLCAhead = 4;

template <class T>
__global__ __launch_bounds__(256) void lincomb_grouped_kernel(const LCGroup* __restrict__ groups,
                                                              const LCTarget* __restrict__ tg,
                                                              const LCSource* __restrict__ us,
                                                              const T* __restrict__ coef, Bases bs0,
                                                              const Bases* __restrict__ ib) {
  constexpr int kElems = lc_elems<T>();
  const LCGroup G = groups[blockIdx.y];
  const Bases& bs = ib ? ib[G.inst] : bs0;
  const long bz = blockIdx.z;
  const long span = long(blockDim.x) * kElems;
  for (long e0 = long(blockIdx.x) * span + threadIdx.x; e0 < G.size; e0 += long(gridDim.x) * span) {
    bool in[kElems];
#pragma unroll
    for (int j = 0; j < kElems; ++j) in[j] = e0 + long(j) * blockDim.x < G.size;
    T acc[kElems][kLCGroup];
#pragma unroll
    for (int j = 0; j < kElems; ++j)
#pragma unroll
      for (int k = 0; k < kLCGroup; ++k) acc[j][k] = T(0);
    int u = G.u0;
    for (; u + kLCAhead <= G.u1; u += kLCAhead) {
      T x[kLCAhead][kElems];
#pragma unroll
      for (int v = 0; v < kLCAhead; ++v) {
        const LCSource q = us[u + v];
        const T* p = reinterpret_cast<const T*>(bs.p[q.base]) + q.off + bz * bs.stride[q.base] + e0;
#pragma unroll
        for (int j = 0; j < kElems; ++j) x[v][j] = in[j] ? p[long(j) * blockDim.x] : T(0);
      }
#pragma unroll
      for (int v = 0; v < kLCAhead; ++v)
#pragma unroll
        for (int k = 0; k < kLCGroup; ++k) {
          const T c = coef[long(u + v) * kLCGroup + k];
#pragma unroll
          for (int j = 0; j < kElems; ++j) acc[j][k] += c * x[v][j];
        }
    }
    for (; u < G.u1; ++u) {
      const LCSource q = us[u];
      const T* p = reinterpret_cast<const T*>(bs.p[q.base]) + q.off + bz * bs.stride[q.base] + e0;
      T x[kElems];
#pragma unroll
      for (int j = 0; j < kElems; ++j) x[j] = in[j] ? p[long(j) * blockDim.x] : T(0);
#pragma unroll
      for (int k = 0; k < kLCGroup; ++k) {
        const T c = coef[long(u) * kLCGroup + k];
#pragma unroll
        for (int j = 0; j < kElems; ++j) acc[j][k] += c * x[j];
      }
    }
#pragma unroll
    for (int k = 0; k < kLCGroup; ++k) {
      if (k < G.nt) {
        const LCTarget t = tg[G.t0 + k];
        T* o = reinterpret_cast<T*>(bs.p[t.base]) + t.off + bz * bs.stride[t.base] + e0;
#pragma unroll
        for (int j = 0; j < kElems; ++j) {
          if (!in[j]) continue;
          T* oj = o + long(j) * blockDim.x;
          *oj = t.accumulate ? *oj + acc[j][k] : acc[j][k];
        }
      }
    }
  }
}

void launch_lincomb_grouped(int prec, const LCGroup* g, int ngroups, const LCTarget* t, const LCSource* u,
                            const double* coef, const float* coef32, long max_size, const Bases& b, int batch,
                            hipStream_t s, const Bases* ib) {
  if (ngroups <= 0 || max_size <= 0 || batch <= 0) return;
  const long span = 256L * (prec == 0 ? lc_elems<double>() : lc_elems<float>());
  long blocks = (max_size + span - 1) / span;
  if (blocks > 1024) blocks = 1024;
  for (int g0 = 0; g0 < ngroups; g0 += 65535) {
    const int ng = ngroups - g0 < 65535 ? ngroups - g0 : 65535;
    const dim3 grid(unsigned(blocks), ng, batch);
    if (prec == 0)
      hipLaunchKernelGGL(lincomb_grouped_kernel<double>, grid, dim3(256), 0, s, g + g0, t, u, coef, b, ib);
    else
      hipLaunchKernelGGL(lincomb_grouped_kernel<float>, grid, dim3(256), 0, s, g + g0, t, u, coef32, b, ib);
  }
}

__global__ void copy2d_kernel(const Copy2D* __restrict__ jobs) {
  const Copy2D J = jobs[blockIdx.y];
  const long n = long(J.rows) * J.cols;
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) {
    const long r = e / J.cols, c = e % J.cols;
    double v = J.src[r * J.ss_r + c * J.ss_c];
    if (J.mode == 1) v *= J.scale[r];
    else if (J.mode == 2) v *= J.scale[c];
    J.dst[r * J.ds_r + c * J.ds_c] = v;
  }
}

void launch_copy2d_f64(const Copy2D* jobs, int njobs, hipStream_t s) {
  for (int j0 = 0; j0 < njobs; j0 += 65535) {
    const int nj = njobs - j0 < 65535 ? njobs - j0 : 65535;
    hipLaunchKernelGGL(copy2d_kernel, dim3(64, nj), dim3(256), 0, s, jobs + j0);
  }
}

void launch_lincomb_f64(const LCTarget* t, int ntargets, const LCSource* src, long max_size, const Bases& b,
                        int batch, hipStream_t s) {
  if (ntargets <= 0 || max_size <= 0 || batch <= 0) return;
  long blocks = (max_size + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  for (int t0 = 0; t0 < ntargets; t0 += 65535) {
    const int nt = ntargets - t0 < 65535 ? ntargets - t0 : 65535;
    hipLaunchKernelGGL(lincomb_f64_kernel, dim3(unsigned(blocks), nt, batch), dim3(256), 0, s, t + t0, src, b);
  }
}

void launch_diag_add_f64(const DiagAdd* d, int n, const Bases& b, int batch, hipStream_t s, const Bases* ib) {
  if (n <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(diag_add_f64_kernel, dim3(n, batch), dim3(256), 0, s, d, b, ib);
}

void launch_fill_f64(double* p, long n, double v, hipStream_t s) {
  if (n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, n, v);
}

void launch_add_f64(const double* x, double* y, long n, hipStream_t s) {
  if (n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(add_f64_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, x, y, n);
}

void launch_fill_f32(float* p, long n, hipStream_t s) {
  if (n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_f32_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, n);
}

void launch_diag_jobs_f64(const DiagJob* j, int n, const DiagTerm* t, const Bases& b, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(diag_jobs_f64_kernel, dim3(n), dim3(256), 0, s, j, t, b);
}

// upper bound of the partial sums of any product of length <= n (the chunk
// grows with n, so the count is not monotone in n): at most 512 while the
// chunk is below its cap, n / 4096 beyond
int gram_parts(long n) {
  const long small = (n + 255) / 256, large = (n + 4095) / 4096;
  return int(std::max<long>(std::min<long>(512, small), large));
}

void launch_gram_f64(const double* A, long lda, int na, const double* B, long ldb, int nb, long n, double* G,
                     int ldg, double* part, double alpha, bool accumulate, hipStream_t s) {
  if (na <= 0 || nb <= 0) return;
  const long chunk = gram_chunk(n);
  const int np = n > 0 ? int((n + chunk - 1) / chunk) : 0;  // <= gram_parts(n)
  if (np > 0)
    hipLaunchKernelGGL(gram_part_kernel, dim3(np), dim3(256), 0, s, A, lda, na, B, ldb, nb, n, chunk, part);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((na * nb + 255) / 256), dim3(256), 0, s, part, np, na, nb, G, ldg,
                     alpha, accumulate ? 1 : 0);
}

void launch_axpby_f64(const double* a, const double* x, long ldx, const double* b, double* y, long ldy, int nvec,
                      long n, hipStream_t s) {
  if (nvec <= 0 || n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(axpby_kernel, dim3(unsigned(blocks), nvec), dim3(256), 0, s, a, x, ldx, b, y, ldy, n);
}

void launch_precond_f64(const double* r, const double* d, const double* w, double* z, int nvec, long n, double eps,
                        hipStream_t s) {
  if (nvec <= 0 || n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(precond_kernel, dim3(unsigned(blocks), nvec), dim3(256), 0, s, r, d, w, z, n, eps);
}

void launch_rotate_f64(const double* X, long ldx, int nin, const double* A, int lda, int nout, double* Y, long ldy,
                       long n, hipStream_t s) {
  if (nout <= 0 || n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(rotate_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, X, ldx, nin, A, lda, nout, Y, ldy, n);
}

void launch_block_scale_f64(const BlockScale* bs, int n, const double* vec, double* data, long stride, int batch,
                            hipStream_t s) {
  if (n <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(block_scale_kernel, dim3(n, batch), dim3(256), 0, s, bs, vec, data, stride);
}

void launch_gep_f64(const double* H, const double* S, int n, double thr, double* w, double* X, int* rank,
                    hipStream_t s) {
  hipLaunchKernelGGL(gep_kernel, dim3(1), dim3(256), 0, s, H, S, n, thr, w, X, rank);
}

}  // namespace dmrg
