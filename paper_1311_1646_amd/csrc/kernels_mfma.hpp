// Matrix-core kernels (kernels_mfma.hip).
#pragma once
#include "kernels.hpp"

namespace dmrg {

// Grouped block GEMM on MFMA.  prec 0: FP64 data and accumulate; 1: FP32
// data, FP32 accumulate; 2: FP32 data split into bfloat16 hi/lo, three
// products, FP32 accumulate.  For prec 1/2 the operands are FP32 and the
// output is FP64 (out_f64) or FP32; bout gives the output base pointers
// (may equal b).
void launch_grouped_gemm(int prec, bool out_f64, const GTile* tiles, int ntiles, const GJob* jobs,
                         const GContrib* con, const Bases& b, const Bases& bout, int batch, hipStream_t s);

void launch_lincomb_f32(const LCTarget* t, int ntargets, const LCSource* src, long max_size, const Bases& b,
                        int batch, hipStream_t s);
void launch_diag_add_f32(const DiagAdd* d, int n, const Bases& b, int batch, hipStream_t s);
void launch_convert_f64_f32(const double* in, float* out, long n, hipStream_t s);

}  // namespace dmrg
