// Grouped block GEMM on the CDNA4 matrix cores (gfx950).
//
// Work lists are those of the FMA kernel (tiles / jobs / contributions with
// base-relative addressing).  A workgroup of four waves owns one 64x64 output
// tile, each wave a 32x32 quarter, and streams every contribution of its job
// through LDS in K-chunks.  The chunks of all contributions form one sequence;
// chunk q+1 is fetched from global memory into registers while chunk q is
// multiplied out of LDS, and LDS is double-buffered, so there is a single
// barrier per chunk.  op() transposition, the contribution's alpha and zero
// fill outside the block (ragged edges) are applied while staging.
//
// Batch folding: when one operand is shared by all batch entries and the
// other operand and the output are batched, the batch is folded into the
// free dimension of the batched operand (fold N: columns (v, j) of
// [B_0 | B_1 | ...]; fold M: rows (v, i) of [A_0; A_1; ...]).  The shared
// operand is then staged once per tile instead of once per batch entry and
// the tiles of a narrow block are filled across entries.  Otherwise grid.y
// enumerates the batch entries.
//
//   FP64   : v_mfma_f64_16x16x4f64, 2x2 per wave, FP64 accumulate
//            (16x16 result: lane l, register r holds row l/16 + 4r, column l%16).
//   FP32   : v_mfma_f32_32x32x2f32, FP32 accumulate (32x32 result: lane l,
//            register r holds row 8(r/4) + 4(l/32) + r%4, column l%32).
//   BF16X3 : each FP32 operand split once, at the LDS store, into
//            x = hi + lo (bfloat16); three v_mfma_f32_32x32x16_bf16 products
//            hi*hi + hi*lo + lo*hi with FP32 accumulate (about 2^-16 relative
//            per product).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "kernels_mfma.hpp"

namespace dmrg {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64, TN = 64, NTH = 256;

template <int MODE> struct Cfg;
template <> struct Cfg<0> {  // FP64
  typedef double T;
  static constexpr int TK = 16;
};
template <> struct Cfg<1> {  // FP32
  typedef float T;
  static constexpr int TK = 32;
};
template <> struct Cfg<2> {  // BF16x3
  typedef float T;
  static constexpr int TK = 32;
};

// LDS images of one chunk.  FP64/FP32: a[i][k], b[j][k] (row per output
// index, padded by one element).  BF16x3: hi and lo parts, rows padded to a
// multiple of 16 bytes so that eight consecutive k load as one 128-bit read.
template <int MODE> struct Lds {
  typedef typename Cfg<MODE>::T T;
  static constexpr int TK = Cfg<MODE>::TK;
  T a[2][TM][TK + 1];
  T b[2][TN][TK + 1];
};
template <> struct Lds<2> {
  static constexpr int TK = 32, LD = TK + 8;
  alignas(16) __bf16 ah[2][TM][LD];
  alignas(16) __bf16 al[2][TM][LD];
  alignas(16) __bf16 bh[2][TN][LD];
  alignas(16) __bf16 bl[2][TN][LD];
};

struct TileMap {
  int v[TM];    // batch entry of each tile row (fold M) or column (fold N)
  int idx[TM];  // row / column index inside the block, -1 outside
};

template <int MODE>
struct Stage {
  typedef typename Cfg<MODE>::T T;
  static constexpr int TK = Cfg<MODE>::TK;
  static constexpr int PER = TM * TK / NTH;  // elements per thread and operand
  static constexpr int RUNS = PER / 4;       // runs of 4 elements contiguous in memory
  T ra[PER], rb[PER];
  // Each thread stages RUNS runs of four elements that are contiguous in
  // memory (run r = tid + r*NTH), so one address and one bounds test serve
  // four loads.  The addresses are resolved once per contribution:
  //   op(A) not transposed (contiguous in k): row r/(TK/4), k 4*(r%(TK/4))+e
  //       -> pa[r] points at (row, k) of the run
  //   op(A) transposed (contiguous in rows): k r/(TM/4), rows 4*(r%(TM/4))+e
  //       -> pa[4r+e] points at each row
  //   op(B) not transposed (contiguous in columns): k r/(TN/4), cols 4*(r%(TN/4))+e
  //       -> pb[4r+e] points at each column
  //   op(B) transposed (contiguous in k): column r/(TK/4), k 4*(r%(TK/4))+e
  //       -> pb[r] points at (column, k) of the run
  //   identity A: ia[r] = block row of the run (or -1)
  const T* pa[PER];
  const T* pb[PER];
  int ia[RUNS];
  long lda, ldb;
  int ck, flags;
  T alpha;

  __device__ __forceinline__ void begin(const GContrib& c, const Bases& bs, const TileMap& rm, const TileMap& cm,
                                        int tid) {
    flags = c.flags;
    ck = c.k;
    lda = c.lda;
    ldb = c.ldb;
    alpha = T(c.alpha);
    const bool ta = c.flags & GC_TRANS_A, tb = c.flags & GC_TRANS_B, aid = c.flags & GC_A_IDENTITY;
#pragma unroll
    for (int q = 0; q < PER; ++q) pa[q] = pb[q] = nullptr;
#pragma unroll
    for (int r = 0; r < RUNS; ++r) ia[r] = -1;
    if (aid) {
#pragma unroll
      for (int r = 0; r < RUNS; ++r) ia[r] = rm.idx[(tid + r * NTH) / (TK / 4)];
    } else {
      const T* A = reinterpret_cast<const T*>(bs.p[c.baseA]) + c.offA;
      const long sa = bs.stride[c.baseA];
      if (!ta) {
#pragma unroll
        for (int r = 0; r < RUNS; ++r) {
          const int run = tid + r * NTH, i = run / (TK / 4), ii = rm.idx[i];
          pa[r] = ii < 0 ? nullptr : A + long(rm.v[i]) * sa + long(ii) * c.lda + 4 * (run % (TK / 4));
        }
      } else {
#pragma unroll
        for (int r = 0; r < RUNS; ++r) {
          const int run = tid + r * NTH;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = 4 * (run % (TM / 4)) + e, ii = rm.idx[i];
            pa[4 * r + e] = ii < 0 ? nullptr : A + long(rm.v[i]) * sa + ii;
          }
        }
      }
    }
    const T* B = reinterpret_cast<const T*>(bs.p[c.baseB]) + c.offB;
    const long sb = bs.stride[c.baseB];
    if (!tb) {
#pragma unroll
      for (int r = 0; r < RUNS; ++r) {
        const int run = tid + r * NTH;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 4 * (run % (TN / 4)) + e, jj = cm.idx[j];
          pb[4 * r + e] = jj < 0 ? nullptr : B + long(cm.v[j]) * sb + jj;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < RUNS; ++r) {
        const int run = tid + r * NTH, j = run / (TK / 4), jj = cm.idx[j];
        pb[r] = jj < 0 ? nullptr : B + long(cm.v[j]) * sb + long(jj) * c.ldb + 4 * (run % (TK / 4));
      }
    }
  }

  // Four contiguous elements starting at p (k indices k..k+3 checked
  // against the contribution's inner length).
  __device__ __forceinline__ void run4(T* dst, const T* p, int k, T scale) const {
    if (p && k + 3 < ck) {
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = p[e] * scale;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = (p && k + e < ck) ? p[e] * scale : T(0);
    }
  }

  // Fetch the K-chunk starting at k0 of the current contribution.
  __device__ __forceinline__ void load(int k0, int tid) {
    const bool ta = flags & GC_TRANS_A, tb = flags & GC_TRANS_B, aid = flags & GC_A_IDENTITY;
    if (aid) {
#pragma unroll
      for (int r = 0; r < RUNS; ++r) {
        const int k = k0 + 4 * ((tid + r * NTH) % (TK / 4));
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[4 * r + e] = (ia[r] >= 0 && ia[r] == k + e && k + e < ck) ? alpha : T(0);
      }
    } else if (!ta) {
#pragma unroll
      for (int r = 0; r < RUNS; ++r) {
        const int k = k0 + 4 * ((tid + r * NTH) % (TK / 4));
        run4(ra + 4 * r, pa[r] ? pa[r] + k0 : nullptr, k, alpha);
      }
    } else {
#pragma unroll
      for (int r = 0; r < RUNS; ++r) {
        const int k = k0 + (tid + r * NTH) / (TM / 4);
        const long off = long(k) * lda;
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[4 * r + e] = (pa[4 * r + e] && k < ck) ? pa[4 * r + e][off] * alpha : T(0);
      }
    }
    if (!tb) {
#pragma unroll
      for (int r = 0; r < RUNS; ++r) {
        const int k = k0 + (tid + r * NTH) / (TN / 4);
        const long off = long(k) * ldb;
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[4 * r + e] = (pb[4 * r + e] && k < ck) ? pb[4 * r + e][off] : T(0);
      }
    } else {
#pragma unroll
      for (int r = 0; r < RUNS; ++r) {
        const int k = k0 + 4 * ((tid + r * NTH) % (TK / 4));
        run4(rb + 4 * r, pb[r] ? pb[r] + k0 : nullptr, k, T(1));
      }
    }
  }

  __device__ __forceinline__ void store(Lds<MODE>& s, int buf, bool ta, bool tb, int tid) const {
#pragma unroll
    for (int r = 0; r < RUNS; ++r) {
      const int run = tid + r * NTH;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (ta) put_a(s, buf, 4 * (run % (TM / 4)) + e, run / (TM / 4), ra[4 * r + e]);
        else put_a(s, buf, run / (TK / 4), 4 * (run % (TK / 4)) + e, ra[4 * r + e]);
        if (tb) put_b(s, buf, run / (TK / 4), 4 * (run % (TK / 4)) + e, rb[4 * r + e]);
        else put_b(s, buf, 4 * (run % (TN / 4)) + e, run / (TN / 4), rb[4 * r + e]);
      }
    }
  }

  __device__ __forceinline__ static void put_a(Lds<MODE>& s, int buf, int i, int k, T v) {
    if constexpr (MODE == 2) {
      const __bf16 h = static_cast<__bf16>(v);
      s.ah[buf][i][k] = h;
      s.al[buf][i][k] = static_cast<__bf16>(v - static_cast<float>(h));
    } else {
      s.a[buf][i][k] = v;
    }
  }
  __device__ __forceinline__ static void put_b(Lds<MODE>& s, int buf, int j, int k, T v) {
    if constexpr (MODE == 2) {
      const __bf16 h = static_cast<__bf16>(v);
      s.bh[buf][j][k] = h;
      s.bl[buf][j][k] = static_cast<__bf16>(v - static_cast<float>(h));
    } else {
      s.b[buf][j][k] = v;
    }
  }
};

template <int MODE> struct Acc;
template <> struct Acc<0> {
  doublex4 c[2][2];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) c[a][b] = doublex4{0, 0, 0, 0};
  }
};
template <> struct Acc<1> {
  floatx16 c;
  __device__ void zero() { c = floatx16{0}; }
};
template <> struct Acc<2> {
  floatx16 c;
  __device__ void zero() { c = floatx16{0}; }
};

// Multiply the first kv (<= TK) K-entries of LDS buffer buf into the wave's
// accumulator; (wm, wn) is the wave's 32x32 quarter.
__device__ __forceinline__ void mma(Acc<0>& acc, const Lds<0>& s, int buf, int kv, int wm, int wn, int lane) {
#pragma unroll
  for (int st = 0; st < Cfg<0>::TK / 4; ++st) {
    if (4 * st >= kv) break;
    const int k = 4 * st + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = s.a[buf][wm + 16 * a + (lane & 15)][k];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = s.b[buf][wn + 16 * b + (lane & 15)][k];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.c[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc.c[a][b], 0, 0, 0);
  }
}

__device__ __forceinline__ void mma(Acc<1>& acc, const Lds<1>& s, int buf, int kv, int wm, int wn, int lane) {
#pragma unroll
  for (int st = 0; st < Cfg<1>::TK / 2; ++st) {
    if (2 * st >= kv) break;
    const int k = 2 * st + (lane >> 5);
    acc.c = __builtin_amdgcn_mfma_f32_32x32x2f32(s.a[buf][wm + (lane & 31)][k], s.b[buf][wn + (lane & 31)][k], acc.c,
                                                 0, 0, 0);
  }
}

__device__ __forceinline__ void mma(Acc<2>& acc, const Lds<2>& s, int buf, int kv, int wm, int wn, int lane) {
#pragma unroll
  for (int st = 0; st < Lds<2>::TK / 16; ++st) {
    if (16 * st >= kv) break;
    const int k = 16 * st + 8 * (lane >> 5);
    const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&s.ah[buf][wm + (lane & 31)][k]);
    const bf16x8 al = *reinterpret_cast<const bf16x8*>(&s.al[buf][wm + (lane & 31)][k]);
    const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&s.bh[buf][wn + (lane & 31)][k]);
    const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&s.bl[buf][wn + (lane & 31)][k]);
    acc.c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc.c, 0, 0, 0);
    acc.c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc.c, 0, 0, 0);
    acc.c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc.c, 0, 0, 0);
  }
}

template <class TOut>
__device__ __forceinline__ void put_out(const Bases& bo, const GJob& J, const TileMap& rm, const TileMap& cm, int fold,
                                        int i, int j, double v) {
  const int ii = rm.idx[i], jj = cm.idx[j];
  if (ii < 0 || jj < 0) return;
  const int vb = fold == 2 ? rm.v[i] : cm.v[j];
  TOut* p = reinterpret_cast<TOut*>(bo.p[J.baseC]) + J.offC + long(vb) * bo.stride[J.baseC] + long(ii) * J.ldc + jj;
  *p = (J.flags & GJ_ACCUMULATE) ? TOut(*p + TOut(v)) : TOut(v);
}

__device__ __forceinline__ void write(const Acc<0>& acc, const Bases& bo, const GJob& J, const TileMap& rm,
                                      const TileMap& cm, int fold, int wm, int wn, int lane, bool) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        put_out<double>(bo, J, rm, cm, fold, wm + 16 * a + (lane >> 4) + 4 * r, wn + 16 * b + (lane & 15),
                        acc.c[a][b][r]);
}

template <int MODE>
__device__ __forceinline__ void write(const Acc<MODE>& acc, const Bases& bo, const GJob& J, const TileMap& rm,
                                      const TileMap& cm, int fold, int wm, int wn, int lane, bool out_f64) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), j = wn + (lane & 31);
    if (out_f64) put_out<double>(bo, J, rm, cm, fold, i, j, acc.c[r]);
    else put_out<float>(bo, J, rm, cm, fold, i, j, acc.c[r]);
  }
}

// Row and column maps of tile (tm, tn) of job J (threads 0..127 fill them;
// the caller synchronizes).  fold: 0 = grid.y enumerates batch entries,
// 1 = batch folded into N, 2 = batch folded into M.
__device__ __forceinline__ void tile_maps(TileMap& rm, TileMap& cm, const GJob& J, int tm, int tn, int fold,
                                          int batch, int tid) {
  if (tid < TM) {
    const int g = tm * TM + tid;
    const int mb = fold == 2 ? J.m * batch : J.m;
    rm.v[tid] = fold == 2 ? g / J.m : (fold == 0 ? int(blockIdx.y) : 0);
    rm.idx[tid] = g < mb ? (fold == 2 ? g % J.m : g) : -1;
  } else if (tid < TM + TN) {
    const int u = tid - TM, g = tn * TN + u;
    const int nb = fold == 1 ? J.n * batch : J.n;
    cm.v[u] = fold == 1 ? g / J.n : (fold == 0 ? int(blockIdx.y) : 0);
    cm.idx[u] = g < nb ? (fold == 1 ? g % J.n : g) : -1;
  }
}

template <class PT>
__device__ __forceinline__ void write_partial(const Acc<0>& acc, PT* P, int wm, int wn, int lane) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        P[(wm + 16 * a + (lane >> 4) + 4 * r) * TN + wn + 16 * b + (lane & 15)] = PT(acc.c[a][b][r]);
}
template <int MODE, class PT>
__device__ __forceinline__ void write_partial(const Acc<MODE>& acc, PT* P, int wm, int wn, int lane) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
    P[(wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * TN + wn + (lane & 31)] = PT(acc.c[r]);
}

// ROLE only tags the instantiation (0: products into a workspace, 1: the
// accumulation into the result), so that profiles separate the two stages.
template <int MODE, int ROLE>
__global__ __launch_bounds__(NTH) void ggemm_mfma_kernel(const GTile* __restrict__ tiles,
                                                         const GJob* __restrict__ jobs,
                                                         const GContrib* __restrict__ con,
                                                         const GSeg* __restrict__ segs, int nslots,
                                                         typename Cfg<MODE>::T* __restrict__ partial, Bases bs,
                                                         Bases bout, int fold, int batch, int out_f64) {
  __shared__ Lds<MODE> s;
  __shared__ TileMap rm, cm;
  __shared__ Bases sb;  // base table indexed per contribution (LDS, not a private copy)
  constexpr int TK = Cfg<MODE>::TK;
  const GTile t = tiles[blockIdx.x];
  const GJob J = jobs[t.job];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  int c0 = J.c0, c1 = J.c1, slot = -1;
  if (t.pad >= 0) {
    const GSeg g = segs[t.pad];
    c0 = g.c0;
    c1 = g.c1;
    slot = g.slot;
  }
  tile_maps(rm, cm, J, t.tm, t.tn, fold, batch, tid);
  if (tid >= TM + TN && tid < TM + TN + kMaxBases) {
    sb.p[tid - TM - TN] = bs.p[tid - TM - TN];
    sb.stride[tid - TM - TN] = bs.stride[tid - TM - TN];
  }
  __syncthreads();
  Acc<MODE> acc;
  acc.zero();
  if (c0 < c1) {
    Stage<MODE> st;
    int ci = c0, k0 = 0, buf = 0;
    st.begin(con[ci], sb, rm, cm, tid);
    st.load(0, tid);
    for (;;) {
      const int ck = st.ck, fl = st.flags;
      st.store(s, buf, fl & GC_TRANS_A, fl & GC_TRANS_B, tid);
      __syncthreads();
      const int kv = ck - k0 < TK ? ck - k0 : TK;
      int nci = ci, nk0 = k0 + TK;
      if (nk0 >= ck) {
        ++nci;
        nk0 = 0;
      }
      const bool more = nci < c1;
      if (more) {
        if (nci != ci) st.begin(con[nci], sb, rm, cm, tid);
        st.load(nk0, tid);
      }
      mma(acc, s, buf, kv, wm, wn, lane);
      if (!more) break;
      ci = nci;
      k0 = nk0;
      buf ^= 1;
    }
  }
  if (slot >= 0) {
    const long entry = fold == 0 ? long(blockIdx.y) : 0;
    write_partial(acc, partial + (entry * nslots + slot) * long(TM * TN), wm, wn, lane);
  } else {
    write(acc, bout, J, rm, cm, fold, wm, wn, lane, out_f64 != 0);
  }
}

// Sum the partial tiles of each reduction item in segment order and write
// the tile to its output block.
template <class PT>
__global__ __launch_bounds__(NTH) void reduce_partials_kernel(const GRed* __restrict__ red,
                                                              const GJob* __restrict__ jobs,
                                                              const PT* __restrict__ partial, int nslots, Bases bout,
                                                              int fold, int batch, int out_f64) {
  __shared__ TileMap rm, cm;
  const GRed r = red[blockIdx.x];
  const GJob J = jobs[r.job];
  const int tid = threadIdx.x;
  tile_maps(rm, cm, J, r.tm, r.tn, fold, batch, tid);
  __syncthreads();
  const long entry = fold == 0 ? long(blockIdx.y) : 0;
  const PT* P = partial + (entry * nslots + r.slot0) * long(TM * TN);
  for (int e = tid; e < TM * TN; e += NTH) {
    const int i = e / TN, j = e % TN;
    if (rm.idx[i] < 0 || cm.idx[j] < 0) continue;
    double sum = 0;
    for (int q = 0; q < r.nseg; ++q) sum += double(P[long(q) * TM * TN + e]);
    if (out_f64) put_out<double>(bout, J, rm, cm, fold, i, j, sum);
    else put_out<float>(bout, J, rm, cm, fold, i, j, sum);
  }
}

__global__ void lincomb_f32_kernel(const LCTarget* __restrict__ tg, const LCSource* __restrict__ src, Bases bs) {
  const LCTarget t = tg[blockIdx.y];
  const int bz = blockIdx.z;
  float* out = reinterpret_cast<float*>(bs.p[t.base]) + t.off + long(bz) * bs.stride[t.base];
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < t.size; e += long(gridDim.x) * blockDim.x) {
    float acc = 0.f;
    for (int j = t.s0; j < t.s1; ++j) {
      const float* p =
          reinterpret_cast<const float*>(bs.p[src[j].base]) + src[j].off + long(bz) * bs.stride[src[j].base];
      acc = fmaf(float(src[j].c), p[e], acc);
    }
    out[e] = t.accumulate ? out[e] + acc : acc;
  }
}

__global__ void diag_add_f32_kernel(const DiagAdd* __restrict__ d, Bases bs) {
  const DiagAdd x = d[blockIdx.x];
  float* o = reinterpret_cast<float*>(bs.p[x.base]) + x.off + long(blockIdx.y) * bs.stride[x.base];
  for (int i = threadIdx.x; i < x.dim; i += blockDim.x) o[long(i) * (x.dim + 1)] += float(x.c);
}

__global__ void convert_f64_f32_kernel(const double* __restrict__ in, float* __restrict__ out, long n) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x)
    out[e] = float(in[e]);
}

}  // namespace

template <int MODE>
void launch_mode(int role, dim3 grid, hipStream_t s, const GTile* tiles, const GJob* jobs, const GContrib* con,
                 const GSeg* segs, int nslots, void* partial, const Bases& b, const Bases& bout, int fold, int batch,
                 int of) {
  typedef typename Cfg<MODE>::T T;
  T* P = static_cast<T*>(partial);
  if (role == 0)
    hipLaunchKernelGGL((ggemm_mfma_kernel<MODE, 0>), grid, dim3(NTH), 0, s, tiles, jobs, con, segs, nslots, P, b, bout,
                       fold, batch, of);
  else
    hipLaunchKernelGGL((ggemm_mfma_kernel<MODE, 1>), grid, dim3(NTH), 0, s, tiles, jobs, con, segs, nslots, P, b, bout,
                       fold, batch, of);
}

void launch_grouped_gemm(int prec, bool out_f64, int role, const GTile* tiles, int ntiles, const GJob* jobs,
                         const GContrib* con, const GSeg* segs, int nslots, void* partial, const Bases& b,
                         const Bases& bout, int fold, int batch, hipStream_t s) {
  if (ntiles <= 0 || batch <= 0) return;
  const dim3 grid(ntiles, fold == 0 ? batch : 1);
  if (prec == 0) launch_mode<0>(role, grid, s, tiles, jobs, con, segs, nslots, partial, b, bout, fold, batch, 1);
  else if (prec == 1)
    launch_mode<1>(role, grid, s, tiles, jobs, con, segs, nslots, partial, b, bout, fold, batch, out_f64 ? 1 : 0);
  else launch_mode<2>(role, grid, s, tiles, jobs, con, segs, nslots, partial, b, bout, fold, batch, out_f64 ? 1 : 0);
}

void launch_reduce_partials(int prec, bool out_f64, const GRed* red, int nred, const GJob* jobs, int nslots,
                            const void* partial, const Bases& bout, int fold, int batch, hipStream_t s) {
  if (nred <= 0 || batch <= 0) return;
  const dim3 grid(nred, fold == 0 ? batch : 1);
  if (prec == 0)
    hipLaunchKernelGGL(reduce_partials_kernel<double>, grid, dim3(NTH), 0, s, red, jobs,
                       static_cast<const double*>(partial), nslots, bout, fold, batch, 1);
  else
    hipLaunchKernelGGL(reduce_partials_kernel<float>, grid, dim3(NTH), 0, s, red, jobs,
                       static_cast<const float*>(partial), nslots, bout, fold, batch, out_f64 ? 1 : 0);
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
