// Device kernel interfaces (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmrg {

// One GEMM contribution C_tile += alpha * op(A) * op(B).
enum : int {
  GC_TRANS_A = 1,
  GC_TRANS_B = 2,
  GC_A_IDENTITY = 4,  // op(A) is the identity (A unused)
  GC_A_BATCHED = 8,   // A advances by the launch's batch stride of A
  GC_B_BATCHED = 16,
  GC_B_BATCHED_ALT = 32,  // B advances by the batch stride of A (second batched space)
};
struct GContrib {
  const void* A;
  const void* B;
  int lda, ldb, k, flags;
  double alpha;
};
enum : int { GJ_ACCUMULATE = 1, GJ_C_BATCHED = 2 };
struct GJob {
  void* C;
  int ldc, m, n;
  int c0, c1;  // contribution range
  int flags;
  int pad;
};
struct GTile {
  int job, tm, tn, pad;
};

// Grouped, tiled GEMM over a list of output tiles; each output tile sums all
// contributions of its job in order (deterministic, no atomics).
// grid.y = batch; batched operands advance by sA/sB/sC elements per batch.
void launch_grouped_gemm_f64(const GTile* tiles, int ntiles, const GJob* jobs, const GContrib* con,
                             int batch, long sA, long sB, long sC, hipStream_t s);

// Linear combinations out_t = [out_t +] sum_j c_j src_j over `size_t` elements.
struct LCTarget {
  double* out;
  long size;
  int s0, s1;  // source range
  int accumulate;
  int pad;
};
struct LCSource {
  const double* src;
  double c;
};
void launch_lincomb_f64(const LCTarget* t, int ntargets, const LCSource* src, long max_size,
                        int batch, long stride, hipStream_t s);

// out[off_k + i*(dim_k+1)] += c for i < dim_k (identity on diagonal blocks)
struct DiagAdd {
  double* out;
  int dim;
  int pad;
  double c;
};
void launch_diag_add_f64(const DiagAdd* d, int n, int maxdim, hipStream_t s);

void launch_fill_f64(double* p, long n, double v, hipStream_t s);

// Diagonal of sum_t alpha_t X_t (x) |n><n| (x) Z_t on one output block:
// out[l, r] (+)= sum_t alpha_t X_t[l, l] Z_t[r, r]; one workgroup per job.
struct DiagTerm {
  const double* X;  // diagonal block of the left operator (rows x rows) or null = identity
  const double* Z;  // diagonal block of the right operator (cols x cols) or null = identity
  double alpha;
};
struct DiagJob {
  double* out;
  int rows, cols;
  int t0, t1;
};
void launch_diag_jobs_f64(const DiagJob* j, int n, const DiagTerm* t, hipStream_t s);

}  // namespace dmrg
