// Device kernel interfaces (implemented in kernels.hip).
//
// All work lists address memory as (base id, element offset): a launch
// receives up to kMaxBases base pointers, each with its own batch stride
// (0 = shared by all batch entries).  Lists are therefore independent of the
// buffers they run on and are built once per site and kind, then reused.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmrg {

constexpr int kMaxBases = 12;

struct Bases {
  double* p[kMaxBases];
  long stride[kMaxBases];
};

enum : int {
  GC_TRANS_A = 1,
  GC_TRANS_B = 2,
  GC_A_IDENTITY = 4,  // op(A) is the identity (A unused)
};

// One contribution C_tile += alpha * op(A) * op(B).
struct GContrib {
  long offA, offB;
  int lda, ldb, k, flags;
  int baseA, baseB;
  double alpha;
};

// Gathered operands: with GJ_GATHER_A row i of op(A) (A not transposed,
// rows contiguous in k) starts at element gather[pad + i] of A's base; with
// GJ_GATHER_B column j of op(B) (B transposed, columns contiguous in k)
// starts at gather[pad + j] of B's base.  The contribution's own offset of
// that operand is then unused (zero).  A job with a gathered operand has one
// contribution: it stacks many small products that share the other operand
// into one matrix, so its tiles are filled across them.
enum : int { GJ_ACCUMULATE = 1, GJ_GATHER_A = 2, GJ_GATHER_B = 4 };
struct GJob {
  long offC;
  int baseC, ldc, m, n;
  int c0, c1;  // contribution range
  int flags, pad;  // pad: start of the job's gather entries
  int inst;        // instance of a grouped launch (index into its base tables)
};
struct GTile {
  int job, tm, tn, pad;
};

// Grouped, tiled GEMM over a list of output tiles; each output tile sums all
// contributions of its job in order (deterministic, no atomics).  grid.y =
// batch entries.
void launch_grouped_gemm_f64(const GTile* tiles, int ntiles, const GJob* jobs, const GContrib* con,
                             const int* gather, const Bases& b, int batch, hipStream_t s);

// Linear combinations out = [out +] sum_j c_j src_j.
struct LCTarget {
  long off, size;
  int base, s0, s1, accumulate;
};
struct LCSource {
  long off;
  int base, pad;
  double c;
};
void launch_lincomb_f64(const LCTarget* t, int ntargets, const LCSource* src, long max_size, const Bases& b,
                        int batch, hipStream_t s);

// Grouped linear combinations: up to kLCGroup targets of equal size read one
// merged, sorted list of sources; each source element is loaded once per
// group and applied to every target of the group with its coefficient
// (coef[u * kLCGroup + k], zero where target k does not use source u).
constexpr int kLCGroup = 16;
struct LCGroup {
  long size;
  int t0, nt, u0, u1;
  int inst;  // instance of a grouped launch
};
// prec 0: FP64 data and coefficients coef; otherwise FP32 data and the
// same coefficients rounded to FP32 (coef32)
void launch_lincomb_grouped(int prec, const LCGroup* g, int ngroups, const LCTarget* t, const LCSource* u,
                            const double* coef, const float* coef32, long max_size, const Bases& b, int batch,
                            hipStream_t s, const Bases* ib = nullptr);

// Strided 2-D copies dst(r, c) = src(r, c) * scale, element (r, c) at
// r*ss_r + c*ss_c in the source and r*ds_r + c*ds_c in the destination;
// mode 0: no scale, 1: scale[r], 2: scale[c].  Jobs are independent.
struct Copy2D {
  const double* src;
  double* dst;
  long ss_r, ss_c, ds_r, ds_c;
  const double* scale;
  int rows, cols, mode, pad;
};
void launch_copy2d_f64(const Copy2D* jobs, int njobs, hipStream_t s);

// out[off + i*(dim+1)] += c for i < dim (identity added to a diagonal block)
struct DiagAdd {
  long off;
  int base, dim;
  double c;
  int inst;  // instance of a grouped launch
};
// ib: per-instance base tables of a grouped launch (indexed by the job's,
// group's or entry's instance), or null: every entry uses b
void launch_diag_add_f64(const DiagAdd* d, int n, const Bases& b, int batch, hipStream_t s,
                         const Bases* ib = nullptr);

void launch_fill_f64(double* p, long n, double v, hipStream_t s);
void launch_fill_f32(float* p, long n, hipStream_t s);  // p[0..n) = 0
void launch_add_f64(const double* x, double* y, long n, hipStream_t s);  // y[0..n) += x[0..n)

// Diagonal of sum_t alpha_t X_t (x) |n><n| (x) Z_t on one output block:
// out[l, r] = sum_t alpha_t X_t[l, l] Z_t[r, r]; one workgroup per job.
struct DiagTerm {
  long offX, offZ;  // -1 = identity
  int baseX, baseZ;
  double alpha;
};
struct DiagJob {
  long off;
  int base, rows, cols, t0, t1, pad;
};
void launch_diag_jobs_f64(const DiagJob* j, int n, const DiagTerm* t, const Bases& b, hipStream_t s);

// ---- dense vector kernels on [nvec][n] arrays (FP64)

// G[m*ldg + k] (+)= alpha * sum_e A[m*lda + e] * B[k*ldb + e]  (m < na, k < nb),
// split over e with a deterministic two-pass reduction (the split depends on
// n only); part must hold gram_parts(n) * na * nb doubles, and
// gram_parts(n) bounds the partial sums of every product of length <= n, so
// a buffer sized for the longest vector serves all shorter ones.
int gram_parts(long n);
void launch_gram_f64(const double* A, long lda, int na, const double* B, long ldb, int nb, long n, double* G,
                     int ldg, double* part, double alpha, bool accumulate, hipStream_t s);

// y[v][e] = a[v] * x[v][e] + b[v] * y[v][e]  (per-vector scalars in device memory)
void launch_axpby_f64(const double* a, const double* x, long ldx, const double* b, double* y, long ldy, int nvec,
                      long n, hipStream_t s);

// z[v][e] = r[v][e] / g(d[e] - w[v]) with g(x) = x if |x| >= eps else +-eps
void launch_precond_f64(const double* r, const double* d, const double* w, double* z, int nvec, long n,
                        double eps, hipStream_t s);

// Y[v][e] = sum_u X[u][e] * A[u + v*lda]  (v < nout, u < nin)
void launch_rotate_f64(const double* X, long ldx, int nin, const double* A, int lda, int nout, double* Y, long ldy,
                       long n, hipStream_t s);

// scale the rows (by_rows) or columns of one block by entries of a vector
struct BlockScale {
  long off, vec_off;
  int rows, cols, by_rows, pad;
};
void launch_block_scale_f64(const BlockScale* bs, int n, const double* vec, double* data, long stride, int batch,
                            hipStream_t s);

// Symmetric generalized eigenproblem H x = w S x (n <= 64) in one workgroup:
// canonical orthogonalization of S (eigenvalues <= thr * max dropped), then
// Jacobi on the projected H.  Ascending w[0..rank), vectors X (column-major,
// leading dimension n; X^T S X = 1 on the kept columns), rank.
void launch_gep_f64(const double* H, const double* S, int n, double thr, double* w, double* X, int* rank,
                    hipStream_t s);

}  // namespace dmrg
