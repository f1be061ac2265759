// Matrix-core kernels (kernels_mfma.hip).
#pragma once
#include "kernels.hpp"

namespace dmrg {

// Grouped block GEMM on MFMA.  prec 0: FP64 data and accumulate; 1: FP32
// data, FP32 accumulate; 2: FP32 data split into bfloat16 hi/lo, three
// products, FP32 accumulate.  For prec 1/2 the operands are FP32 and the
// output is FP64 (out_f64) or FP32; bout gives the output base pointers
// (may equal b).  fold 0: grid.y runs over the batch entries and the tiles
// are (job, row tile, column tile) of each job's m x n; fold 1 (B and C
// batched, A shared): tiles cover m x (batch*n); fold 2 (A and C batched, B
// shared): tiles cover (batch*m) x n.
//
// Split contribution lists: a tile whose `pad` field is >= 0 handles only the
// contribution range of segs[pad] and writes its dense 64x64 partial sum to
// slot `slot` of the partial buffer (per batch entry when fold is 0: slot +
// entry * nslots).  A second kernel then sums the nseg partials of each
// reduction item in order and writes the tile to the output (deterministic,
// no atomics).
enum : int { FOLD_NONE = 0, FOLD_N = 1, FOLD_M = 2 };
struct GSeg {
  int c0, c1, slot, pad;
};
struct GRed {
  int job, tm, tn, slot0, nseg, pad;
};
// Output tile shapes of the matrix-core kernel (rows x columns).  128x128
// (512-thread workgroups) exists for FP32 and BF16x3 operands only.
enum : int { TILE_64x64 = 0, TILE_128x64 = 1, TILE_64x128 = 2, TILE_128x128 = 3 };
int tile_rows(int shape);
int tile_cols(int shape);

// role 0: products into a workspace, 1: accumulation into the result (the
// two instantiations are the same code; the tag separates them in profiles).
// Tiles index shape-sized tiles; partial slots hold dense rows x columns
// tiles of the operand type.
// gather: entries of the jobs with a gathered operand (may be null when no
// job has one).
// ib: per-instance base tables of a grouped launch (GJob::inst selects one;
// the outputs are written through it too), or null (b and bout for all).
void launch_grouped_gemm(int prec, bool out_f64, int role, int shape, const GTile* tiles, int ntiles,
                         const GJob* jobs, const GContrib* con, const int* gather, const GSeg* segs, int nslots,
                         void* partial, const Bases& b, const Bases& bout, int fold, int batch, hipStream_t s,
                         const Bases* ib = nullptr);
void launch_reduce_partials(int prec, bool out_f64, int shape, const GRed* red, int nred, const GJob* jobs,
                            int nslots, const void* partial, const Bases& bout, int fold, int batch, hipStream_t s,
                            const Bases* ib = nullptr);

void launch_diag_add_f32(const DiagAdd* d, int n, const Bases& b, int batch, hipStream_t s,
                         const Bases* ib = nullptr);
void launch_convert_f64_f32(const double* in, float* out, long n, hipStream_t s);
// several FP64 -> FP32 conversions in one launch (grid.y = jobs)
struct ConvJob {
  const double* in;
  float* out;
  long n;
};
void launch_convert_list(const ConvJob* jobs, int njobs, long max_n, hipStream_t s);

}  // namespace dmrg
