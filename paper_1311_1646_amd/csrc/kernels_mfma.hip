// Grouped block GEMM on the CDNA4 matrix cores (gfx950).
//
// Work lists are those of the FMA kernel (tiles / jobs / contributions with
// base-relative addressing).  A workgroup of four waves owns one TM x TN
// output tile (64x64, 128x64 or 64x128), each wave a (TM/2) x (TN/2)
// quarter, and streams every contribution of its job through LDS in
// K-chunks.  The chunks of all contributions form one sequence; chunk q+1 is
// fetched from global memory into registers while chunk q is multiplied out
// of LDS, and LDS is double-buffered, so there is a single barrier per chunk.
// op() transposition, the contribution's alpha and zero fill outside the
// block (ragged edges) are applied while staging.
//
// Batch folding: when one operand is shared by all batch entries and the
// other operand and the output are batched, the batch is folded into the
// free dimension of the batched operand (fold N: columns (v, j) of
// [B_0 | B_1 | ...]; fold M: rows (v, i) of [A_0; A_1; ...]).  The shared
// operand is then staged once per tile instead of once per batch entry and
// the tiles of a narrow block are filled across entries.  Otherwise grid.y
// enumerates the batch entries.  The 128-wide tile shapes put 128 along the
// unfolded (block) dimension, so a symmetry block of up to 128 rows or
// columns is covered by one tile and the batched operand is read once.
//
//   FP64   : v_mfma_f64_16x16x4f64, FP64 accumulate
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

constexpr int NTH = 256;  // threads of the auxiliary kernels

// Workgroup geometry of a TM x TN output tile: 256 threads (four waves in
// 2 x 2) up to 128 x 64, 512 threads (eight waves in 2 x 4) for 128 x 128, so
// that every thread stages the same four elements of each operand per
// K-chunk while a wave's share of the matrix-core work doubles.  Each wave
// owns a (TM / 2) x (TN / WN) part of the tile.
template <int TM, int TN> struct Geo {
  static constexpr int NT = TM * TN >= 128 * 128 ? 512 : 256;
  static constexpr int WN = NT / 128;  // waves along N (two along M)
  static constexpr int WTM = TM / 2, WTN = TN / WN;
};

template <int MODE> struct Cfg;
template <> struct Cfg<0> {  // FP64
  typedef double T;
  static constexpr int TK = 16, MB = 16;  // K-chunk, side of one MFMA result block
};
template <> struct Cfg<1> {  // FP32
  typedef float T;
  static constexpr int TK = 16, MB = 32;
};
template <> struct Cfg<2> {  // BF16x3
  typedef float T;
  static constexpr int TK = 16, MB = 32;
};

// LDS images of one chunk, one row per output index (tile row of op(A),
// tile column of op(B)), written four consecutive k at a time.
//   FP64  : a[i][k], rows padded by one element.
//   FP32  : a[i][p(k)] with p(k) = 8 (k & 1) + (k >> 1) (K-chunks of 16):
//           the 32x32x2 product at step s takes k = 2s + h in lane half h,
//           so the eight values a lane needs over a chunk are contiguous
//           (two 128-bit reads); rows padded to 20 elements (16-byte
//           aligned).
//   BF16x3: hi and lo parts, k contiguous (K-chunks of 16, one 32x32x16
//           product per part pair), rows padded to a multiple of 16 bytes so
//           that eight consecutive k load as one 128-bit read.
template <int MODE, int TM, int TN> struct Lds {
  typedef typename Cfg<MODE>::T T;
  static constexpr int TK = Cfg<MODE>::TK;
  T a[2][TM][TK + 1];
  T b[2][TN][TK + 1];
};
// Rows of the output tile transposed through LDS per pass (write_rows).
template <int TM, int TN> struct OutPass {
  static constexpr int ROWS = TM * TN >= 128 * 128 ? TM / 2 : TM;
};
template <int TM, int TN> struct Lds<1, TM, TN> {
  static constexpr int TK = 16, LD = TK + 4;
  alignas(16) float a[2][TM][LD];
  alignas(16) float b[2][TN][LD];
  // the finished tile is transposed through this storage (ROWS x (TN + 8))
  static constexpr int O = OutPass<TM, TN>::ROWS * (TN + 8);
  float spare[O > 2 * (TM + TN) * LD ? O - 2 * (TM + TN) * LD : 1];
};
template <int TM, int TN> struct Lds<2, TM, TN> {
  static constexpr int TK = 16, LD = TK + 8;
  alignas(16) __bf16 ah[2][TM][LD];
  alignas(16) __bf16 al[2][TM][LD];
  alignas(16) __bf16 bh[2][TN][LD];
  alignas(16) __bf16 bl[2][TN][LD];
};

template <int TM, int TN> struct TileMap {
  int rv[TM], ri[TM];  // batch entry / block row of each tile row (-1 outside)
  int cv[TN], cj[TN];  // batch entry / block column of each tile column
  int ga[TM], gb[TN];  // gathered row / column offsets (jobs with a gathered operand)
};

// Global-memory pointers: loads through them are global loads (counted by
// vmcnt only), not flat loads that would also hold up the LDS waits of the
// multiply while the next chunk is in flight.
template <class T> using gptr = const __attribute__((address_space(1))) T*;

// Four consecutive k (k0 a multiple of 4) of one LDS row.
__device__ __forceinline__ void put4_f32(float* rowp, int k0, const float* v) {
  // p(k0) = k0/2 (even k), p(k0 + 1) = 8 + k0/2 (odd k)
  *reinterpret_cast<float2*>(rowp + (k0 >> 1)) = float2{v[0], v[2]};
  *reinterpret_cast<float2*>(rowp + 8 + (k0 >> 1)) = float2{v[1], v[3]};
}
__device__ __forceinline__ void put4_bf16(__bf16* hip, __bf16* lop, int k0, const float* v) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  bf16x4 h, l;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    h[e] = static_cast<__bf16>(v[e]);
    l[e] = static_cast<__bf16>(v[e] - static_cast<float>(h[e]));
  }
  *reinterpret_cast<bf16x4*>(hip + k0) = h;
  *reinterpret_cast<bf16x4*>(lop + k0) = l;
}

// Staging of one K-chunk of op(A) (TM x TK) and op(B) (TK x TN).  Each
// thread holds TM*TK/NTH (resp. TN*TK/NTH) elements as runs of four
// consecutive k of one row, in one of two maps:
//   k-map   (operand contiguous in k: A not transposed, B transposed,
//            identity A): run q = tid + q*NTH covers row q/(TK/4),
//            k 4*(q%(TK/4)) .. +3; one pointer per run, one wide load.
//   row-map (operand contiguous along the tile: A transposed, B not
//            transposed): the thread owns row u = tid % T and the runs
//            k = 4g + 4Gq .. +3 with g = tid / T, G = NTH / T; one pointer
//            per thread, lanes of a wave read consecutive addresses.
// op() transposition, alpha and the zero fill outside the block are applied
// here; rows outside the block have a null pointer.
template <int MODE, int TM, int TN>
struct Stage {
  typedef typename Cfg<MODE>::T T;
  static constexpr int TK = Cfg<MODE>::TK;
  static constexpr int NTH = Geo<TM, TN>::NT;
  static constexpr int RA = TM * TK / NTH / 4;  // runs per thread, op(A)
  static constexpr int RB = TN * TK / NTH / 4;  // and op(B)
  static constexpr int GA = NTH / TM, GB = NTH / TN;
  static_assert(RA >= 1 && RB >= 1, "fewer than one run of four k per thread");
  static constexpr int NA = 4 * RA, NB = 4 * RB;  // staged elements per thread
  gptr<T> pa[RA];
  gptr<T> pb[RB];
  int ia[RA];
  long lda, ldb;
  int ck, flags;
  T alpha;

  __device__ __forceinline__ void begin(const GContrib& c, const Bases& bs, const TileMap<TM, TN>& m, int tid,
                                        int jflags) {
    flags = c.flags;
    ck = c.k;
    lda = c.lda;
    ldb = c.ldb;
    alpha = T(c.alpha);
    const bool ta = c.flags & GC_TRANS_A, tb = c.flags & GC_TRANS_B, aid = c.flags & GC_A_IDENTITY;
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      pa[q] = nullptr;
      ia[q] = -1;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) pb[q] = nullptr;
    if (aid) {
#pragma unroll
      for (int q = 0; q < RA; ++q) ia[q] = m.ri[(tid + q * NTH) / (TK / 4)];
    } else {
      const gptr<T> A = (gptr<T>)(bs.p[c.baseA]) + c.offA;
      const long sa = bs.stride[c.baseA];
      if (!ta) {
#pragma unroll
        for (int q = 0; q < RA; ++q) {
          const int run = tid + q * NTH, i = run / (TK / 4), ii = m.ri[i];
          const long ro = (jflags & GJ_GATHER_A) ? long(m.ga[i]) : long(ii) * c.lda;
          pa[q] = ii < 0 ? nullptr : A + long(m.rv[i]) * sa + ro + 4 * (run % (TK / 4));
        }
      } else {
        const int u = tid % TM, ii = m.ri[u];
        pa[0] = ii < 0 ? nullptr : A + long(m.rv[u]) * sa + ii;
      }
    }
    const gptr<T> B = (gptr<T>)(bs.p[c.baseB]) + c.offB;
    const long sb = bs.stride[c.baseB];
    if (!tb) {
      const int u = tid % TN, jj = m.cj[u];
      pb[0] = jj < 0 ? nullptr : B + long(m.cv[u]) * sb + jj;
    } else {
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int run = tid + q * NTH, j = run / (TK / 4), jj = m.cj[j];
        const long co = (jflags & GJ_GATHER_B) ? long(m.gb[j]) : long(jj) * c.ldb;
        pb[q] = jj < 0 ? nullptr : B + long(m.cv[j]) * sb + co + 4 * (run % (TK / 4));
      }
    }
  }

  // k-map run: four contiguous elements at p (k .. k+3 checked against the
  // inner length).
  __device__ __forceinline__ void run4(T* dst, gptr<T> p, int k, T scale) const {
    if (p && k + 3 < ck) {
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = p[e] * scale;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = (p && k + e < ck) ? p[e] * scale : T(0);
    }
  }
  // row-map run: elements k .. k+3 of the row at p (stride ld between k);
  // k is the same for every lane of a wave.
  __device__ __forceinline__ void col4(T* dst, gptr<T> p, int k, long ld, T scale) const {
    if (p) {
      const gptr<T> q = p + long(k) * ld;
      if (k + 3 < ck) {
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = q[long(e) * ld] * scale;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = k + e < ck ? q[long(e) * ld] * scale : T(0);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = T(0);
    }
  }

  // Fetch the K-chunk starting at k0 of the current contribution into the
  // thread's staging registers ra (op(A)) and rb (op(B)).
  __device__ __forceinline__ void load(int k0, int tid, T* ra, T* rb) const {
    const bool ta = flags & GC_TRANS_A, tb = flags & GC_TRANS_B, aid = flags & GC_A_IDENTITY;
    if (aid) {
#pragma unroll
      for (int q = 0; q < RA; ++q) {
        const int k = k0 + 4 * ((tid + q * NTH) % (TK / 4));
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[4 * q + e] = (ia[q] >= 0 && ia[q] == k + e && k + e < ck) ? alpha : T(0);
      }
    } else if (!ta) {
#pragma unroll
      for (int q = 0; q < RA; ++q) {
        const int k = k0 + 4 * ((tid + q * NTH) % (TK / 4));
        run4(ra + 4 * q, pa[q] ? pa[q] + k0 : nullptr, k, alpha);
      }
    } else {
      // tid / TM is the same for all lanes of a wave (TM is a multiple of 64)
      const int g = __builtin_amdgcn_readfirstlane(tid / TM);
#pragma unroll
      for (int q = 0; q < RA; ++q) col4(ra + 4 * q, pa[0], k0 + 4 * g + 4 * GA * q, lda, alpha);
    }
    if (!tb) {
      const int g = __builtin_amdgcn_readfirstlane(tid / TN);
#pragma unroll
      for (int q = 0; q < RB; ++q) col4(rb + 4 * q, pb[0], k0 + 4 * g + 4 * GB * q, ldb, T(1));
    } else {
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int k = k0 + 4 * ((tid + q * NTH) % (TK / 4));
        run4(rb + 4 * q, pb[q] ? pb[q] + k0 : nullptr, k, T(1));
      }
    }
  }

  // Write staged registers of a chunk whose contribution had flags fl.
  __device__ __forceinline__ static void store(Lds<MODE, TM, TN>& s, int buf, int fl, int tid, const T* ra,
                                               const T* rb) {
    const bool ta = fl & GC_TRANS_A, tb = fl & GC_TRANS_B;
    const bool arow = ta && !(fl & GC_A_IDENTITY);
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int run = tid + q * NTH;
      const int row = arow ? tid % TM : run / (TK / 4);
      const int k0 = arow ? 4 * (tid / TM) + 4 * GA * q : 4 * (run % (TK / 4));
      put_a(s, buf, row, k0, ra + 4 * q);
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int run = tid + q * NTH;
      const int row = tb ? run / (TK / 4) : tid % TN;
      const int k0 = tb ? 4 * (run % (TK / 4)) : 4 * (tid / TN) + 4 * GB * q;
      put_b(s, buf, row, k0, rb + 4 * q);
    }
  }

  __device__ __forceinline__ static void put_a(Lds<MODE, TM, TN>& s, int buf, int row, int k0, const T* v) {
    if constexpr (MODE == 2) put4_bf16(&s.ah[buf][row][0], &s.al[buf][row][0], k0, v);
    else if constexpr (MODE == 1) put4_f32(&s.a[buf][row][0], k0, v);
    else {
#pragma unroll
      for (int e = 0; e < 4; ++e) s.a[buf][row][k0 + e] = v[e];
    }
  }
  __device__ __forceinline__ static void put_b(Lds<MODE, TM, TN>& s, int buf, int row, int k0, const T* v) {
    if constexpr (MODE == 2) put4_bf16(&s.bh[buf][row][0], &s.bl[buf][row][0], k0, v);
    else if constexpr (MODE == 1) put4_f32(&s.b[buf][row][0], k0, v);
    else {
#pragma unroll
      for (int e = 0; e < 4; ++e) s.b[buf][row][k0 + e] = v[e];
    }
  }
};

// Accumulators of one wave: BM x BN result blocks of MB x MB.
template <int MODE, int BM, int BN> struct Acc {
  floatx16 c[BM][BN];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b) c[a][b] = floatx16{0};
  }
  // row / column (inside the block) of register r of lane l
  __device__ static int row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  __device__ static int col(int l, int) { return l & 31; }
  static constexpr int R = 16;
};
template <int BM, int BN> struct Acc<0, BM, BN> {
  doublex4 c[BM][BN];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b) c[a][b] = doublex4{0, 0, 0, 0};
  }
  __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
  __device__ static int col(int l, int) { return l & 15; }
  static constexpr int R = 4;
};

// Multiply the first kv (<= TK) K-entries of LDS buffer buf into the wave's
// accumulators; (wm, wn) is the corner of the wave's part of the tile.
template <int TM, int TN, int BM, int BN>
__device__ __forceinline__ void mma(Acc<0, BM, BN>& acc, const Lds<0, TM, TN>& s, int buf, int kv, int wm, int wn,
                                    int lane) {
#pragma unroll
  for (int st = 0; st < Cfg<0>::TK / 4; ++st) {
    if (4 * st >= kv) break;
    const int k = 4 * st + (lane >> 4);
    double av[BM], bv[BN];
#pragma unroll
    for (int a = 0; a < BM; ++a) av[a] = s.a[buf][wm + 16 * a + (lane & 15)][k];
#pragma unroll
    for (int b = 0; b < BN; ++b) bv[b] = s.b[buf][wn + 16 * b + (lane & 15)][k];
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b)
        acc.c[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc.c[a][b], 0, 0, 0);
  }
}

template <int TM, int TN, int BM, int BN>
__device__ __forceinline__ void mma(Acc<1, BM, BN>& acc, const Lds<1, TM, TN>& s, int buf, int kv, int wm, int wn,
                                    int lane) {
  typedef float floatx4 __attribute__((ext_vector_type(4)));
  // all eight steps of the chunk are read first (lane half h holds
  // k = 2s + h at position 8h + s), then the products run back to back
  const int h = 8 * (lane >> 5);
  floatx4 av[BM][2], bv[BN][2];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      av[a][c] = *reinterpret_cast<const floatx4*>(&s.a[buf][wm + 32 * a + (lane & 31)][h + 4 * c]);
#pragma unroll
  for (int b = 0; b < BN; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      bv[b][c] = *reinterpret_cast<const floatx4*>(&s.b[buf][wn + 32 * b + (lane & 31)][h + 4 * c]);
  // groups of four steps (8 k); k beyond the chunk's length is zero in LDS
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (8 * c < kv) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int a = 0; a < BM; ++a)
#pragma unroll
          for (int b = 0; b < BN; ++b)
            acc.c[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a][c][e], bv[b][c][e], acc.c[a][b], 0, 0, 0);
    }
  }
}

template <int TM, int TN, int BM, int BN>
__device__ __forceinline__ void mma(Acc<2, BM, BN>& acc, const Lds<2, TM, TN>& s, int buf, int kv, int wm, int wn,
                                    int lane) {
#pragma unroll
  for (int st = 0; st < Cfg<2>::TK / 16; ++st) {
    if (16 * st >= kv) break;
    const int k = 16 * st + 8 * (lane >> 5);
    bf16x8 ah[BM], al[BM], bh[BN], bl[BN];
#pragma unroll
    for (int a = 0; a < BM; ++a) {
      ah[a] = *reinterpret_cast<const bf16x8*>(&s.ah[buf][wm + 32 * a + (lane & 31)][k]);
      al[a] = *reinterpret_cast<const bf16x8*>(&s.al[buf][wm + 32 * a + (lane & 31)][k]);
    }
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      bh[b] = *reinterpret_cast<const bf16x8*>(&s.bh[buf][wn + 32 * b + (lane & 31)][k]);
      bl[b] = *reinterpret_cast<const bf16x8*>(&s.bl[buf][wn + 32 * b + (lane & 31)][k]);
    }
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b) {
        acc.c[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc.c[a][b], 0, 0, 0);
        acc.c[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc.c[a][b], 0, 0, 0);
        acc.c[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc.c[a][b], 0, 0, 0);
      }
  }
}

template <class TOut, int TM, int TN>
__device__ __forceinline__ void put_out(const Bases& bo, const GJob& J, const TileMap<TM, TN>& m, int fold, int i,
                                        int j, double v) {
  const int ii = m.ri[i], jj = m.cj[j];
  if (ii < 0 || jj < 0) return;
  const int vb = fold == 2 ? m.rv[i] : m.cv[j];
  TOut* p = reinterpret_cast<TOut*>(bo.p[J.baseC]) + J.offC + long(vb) * bo.stride[J.baseC] + long(ii) * J.ldc + jj;
  *p = (J.flags & GJ_ACCUMULATE) ? TOut(*p + TOut(v)) : TOut(v);
}

template <int MODE, int TM, int TN, int BM, int BN>
__device__ __forceinline__ void write(const Acc<MODE, BM, BN>& acc, const Bases& bo, const GJob& J,
                                      const TileMap<TM, TN>& m, int fold, int wm, int wn, int lane, bool out_f64) {
  typedef Acc<MODE, BM, BN> A;
  constexpr int MB = Cfg<MODE>::MB;
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int r = 0; r < A::R; ++r) {
        const int i = wm + MB * a + A::row(lane, r), j = wn + MB * b + A::col(lane, r);
        if (MODE == 0 || out_f64) put_out<double>(bo, J, m, fold, i, j, acc.c[a][b][r]);
        else put_out<float>(bo, J, m, fold, i, j, acc.c[a][b][r]);
      }
}

// FP32 accumulators: the finished tile is transposed through LDS (the
// staging buffers, free once every wave has multiplied its last chunk) so
// that each thread writes runs of four consecutive columns of one output
// row with one address; runs that leave the block or cross a batch entry
// fall back to single elements.
template <class TOut, int MODE, int TM, int TN, int BM, int BN>
__device__ __forceinline__ void write_rows(const Acc<MODE, BM, BN>& acc, float* O, const Bases& bo, const GJob& J,
                                          const TileMap<TM, TN>& m, int fold, int wm, int wn, int lane, int tid) {
  typedef Acc<MODE, BM, BN> A;
  constexpr int MB = Cfg<MODE>::MB, LDO = TN + 8, NT = Geo<TM, TN>::NT, PR = OutPass<TM, TN>::ROWS;
  typedef float floatx4 __attribute__((ext_vector_type(4)));
  const int c4 = 4 * (tid % (TN / 4));
  const int j0 = m.cj[c4], v0 = m.cv[c4];
  const bool run = j0 >= 0 && m.cj[c4 + 3] == j0 + 3 && m.cv[c4 + 3] == v0;
  const long sc = bo.stride[J.baseC];
  TOut* const C = reinterpret_cast<TOut*>(bo.p[J.baseC]) + J.offC;
  const bool accumulate = J.flags & GJ_ACCUMULATE;
#pragma unroll
  for (int pass = 0; pass < TM / PR; ++pass) {
    __syncthreads();
    if (wm >= pass * PR && wm < (pass + 1) * PR) {
#pragma unroll
      for (int a = 0; a < BM; ++a)
#pragma unroll
        for (int b = 0; b < BN; ++b)
#pragma unroll
          for (int r = 0; r < A::R; ++r)
            O[(wm - pass * PR + MB * a + A::row(lane, r)) * LDO + wn + MB * b + A::col(lane, r)] = acc.c[a][b][r];
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PR * TN / 4 / NT; ++p) {
      const int lr = tid / (TN / 4) + p * (NT / (TN / 4));
      const int row = pass * PR + lr;
      const int ii = m.ri[row];
      if (ii < 0) continue;
      const floatx4 v = *reinterpret_cast<const floatx4*>(&O[lr * LDO + c4]);
      if (run) {
        const int vb = fold == 2 ? m.rv[row] : v0;
        TOut* q = C + long(vb) * sc + long(ii) * J.ldc + j0;
        if (accumulate) {
#pragma unroll
          for (int e = 0; e < 4; ++e) q[e] = TOut(q[e] + TOut(v[e]));
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) q[e] = TOut(v[e]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) put_out<TOut, TM, TN>(bo, J, m, fold, row, c4 + e, v[e]);
      }
    }
  }
}

template <int MODE, int TN, int BM, int BN, class PT>
__device__ __forceinline__ void write_partial(const Acc<MODE, BM, BN>& acc, PT* P, int wm, int wn, int lane) {
  typedef Acc<MODE, BM, BN> A;
  constexpr int MB = Cfg<MODE>::MB;
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int r = 0; r < A::R; ++r)
        P[(wm + MB * a + A::row(lane, r)) * TN + wn + MB * b + A::col(lane, r)] = PT(acc.c[a][b][r]);
}

// Row and column maps of tile (tm, tn) of job J (threads 0..TM+TN-1 fill
// them; the caller synchronizes).  fold: 0 = grid.y enumerates batch
// entries, 1 = batch folded into N, 2 = batch folded into M.
template <int TM, int TN>
__device__ __forceinline__ void tile_maps(TileMap<TM, TN>& m, const GJob& J, int tm, int tn, int fold, int batch,
                                          int tid, const int* __restrict__ gather) {
  if (tid < TM) {
    const int g = tm * TM + tid;
    const int mb = fold == 2 ? J.m * batch : J.m;
    const int ri = g < mb ? (fold == 2 ? g % J.m : g) : -1;
    m.rv[tid] = fold == 2 ? g / J.m : (fold == 0 ? int(blockIdx.y) : 0);
    m.ri[tid] = ri;
    m.ga[tid] = (gather && (J.flags & GJ_GATHER_A) && ri >= 0) ? gather[J.pad + ri] : 0;
  } else if (tid < TM + TN) {
    const int u = tid - TM, g = tn * TN + u;
    const int nb = fold == 1 ? J.n * batch : J.n;
    const int cj = g < nb ? (fold == 1 ? g % J.n : g) : -1;
    m.cv[u] = fold == 1 ? g / J.n : (fold == 0 ? int(blockIdx.y) : 0);
    m.cj[u] = cj;
    m.gb[u] = (gather && (J.flags & GJ_GATHER_B) && cj >= 0) ? gather[J.pad + cj] : 0;
  }
}

// One output tile: all contributions of its job (or of its segment) through
// the double-buffered LDS pipeline, then the result or the partial sum.
template <int MODE, int TM, int TN>
__device__ __forceinline__ void do_tile(int ti, const GTile* __restrict__ tiles, const GJob* __restrict__ jobs,
                                        const GContrib* __restrict__ con, const int* __restrict__ gather,
                                        const GSeg* __restrict__ segs, int nslots,
                                        typename Cfg<MODE>::T* __restrict__ partial, int fold, int batch,
                                        int out_f64, Lds<MODE, TM, TN>& s, TileMap<TM, TN>& m, Bases& sb,
                                        const Bases& so, const Bases* __restrict__ ib) {
  constexpr int TK = Cfg<MODE>::TK, MB = Cfg<MODE>::MB;
  typedef Geo<TM, TN> G;
  constexpr int BM = G::WTM / MB, BN = G::WTN / MB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / G::WN) * G::WTM, wn = (wave % G::WN) * G::WTN;
  const GTile t = tiles[ti];
  const GJob J = jobs[t.job];
  int c0 = J.c0, c1 = J.c1, slot = -1;
  if (t.pad >= 0) {
    const GSeg g = segs[t.pad];
    c0 = g.c0;
    c1 = g.c1;
    slot = g.slot;
  }
  // the first contribution's record is requested before the maps are
  // built, so that its latency overlaps theirs and the barrier
  GContrib cfirst{};
  if (c0 < c1) cfirst = con[c0];
  // a grouped launch reads the job's instance table into LDS (after the
  // descriptor loads above are under way) and also writes through it; a
  // plain launch has both tables in LDS already
  if (ib && tid < kMaxBases) {
    sb.p[tid] = ib[J.inst].p[tid];
    sb.stride[tid] = ib[J.inst].stride[tid];
  }
  const Bases& bo = ib ? sb : so;
  tile_maps<TM, TN>(m, J, t.tm, t.tn, fold, batch, tid, gather);
  __syncthreads();
  Acc<MODE, BM, BN> acc;
  acc.zero();
  if (c0 < c1) {
    // The pointer state follows the fetch cursor: chunk q+1 is fetched into
    // the staging registers while chunk q is multiplied out of LDS.  (A
    // second set of registers, two chunks in flight, measured no faster on
    // the FP32 accumulation stage and cost one wave per SIMD.)
    typedef Stage<MODE, TM, TN> St;
    typedef typename Cfg<MODE>::T T;
    St st;
    T ra[St::NA], rb[St::NB];
    int kv = 0, fl = 0;     // valid k of the staged chunk (0: none) and its flags
    int fci = c0, fk = 0;   // next chunk to fetch
    st.begin(cfirst, sb, m, tid, J.flags);
    auto fetch = [&]() {
      if (fci >= c1) {
        kv = 0;
        return;
      }
      st.load(fk, tid, ra, rb);
      kv = st.ck - fk < TK ? st.ck - fk : TK;
      fl = st.flags;
      fk += TK;
      if (fk >= st.ck) {
        ++fci;
        fk = 0;
        if (fci < c1) st.begin(con[fci], sb, m, tid, J.flags);
      }
    };
    fetch();
    int buf = 0;
    while (kv > 0) {
      St::store(s, buf, fl, tid, ra, rb);
      __syncthreads();
      const int kq = kv;
      fetch();
      mma<TM, TN, BM, BN>(acc, s, buf, kq, wm, wn, lane);
      buf ^= 1;
    }
  }
  if (slot >= 0) {
    const long entry = fold == 0 ? long(blockIdx.y) : 0;
    write_partial<MODE, TN>(acc, partial + (entry * nslots + slot) * long(TM * TN), wm, wn, lane);
  } else if constexpr (MODE == 0) {
    write<MODE, TM, TN>(acc, bo, J, m, fold, wm, wn, lane, true);
  } else {
    static_assert(sizeof(Lds<MODE, TM, TN>) >= sizeof(float) * OutPass<TM, TN>::ROWS * (TN + 8),
                  "output pass does not fit");
    float* O = reinterpret_cast<float*>(&s);
    if (out_f64) write_rows<double, MODE, TM, TN>(acc, O, bo, J, m, fold, wm, wn, lane, tid);
    else write_rows<float, MODE, TM, TN>(acc, O, bo, J, m, fold, wm, wn, lane, tid);
  }
}

// Persistent workgroups (a grid of a few rounds of the resident capacity,
// each looping over tiles) pay the launch of a workgroup once; they are used
// where the loop does not cost registers (FP64, capped at 4 waves per SIMD).
template <int MODE> struct Persist {
  static constexpr bool on = MODE == 0;
  static constexpr int waves = MODE == 0 ? 4 : 1;
};

// ROLE only tags the instantiation (0: products into a workspace, 1: the
// accumulation into the result), so that profiles separate the two stages.
template <int MODE, int ROLE, int TM, int TN>
__global__ __launch_bounds__((Geo<TM, TN>::NT), Persist<MODE>::waves) void ggemm_mfma_kernel(
    const GTile* __restrict__ tiles, int ntiles, const GJob* __restrict__ jobs, const GContrib* __restrict__ con,
    const int* __restrict__ gather, const GSeg* __restrict__ segs, int nslots, typename Cfg<MODE>::T* __restrict__ partial, Bases bs, Bases bout,
    int fold, int batch, int out_f64, const Bases* __restrict__ ib) {
  __shared__ Lds<MODE, TM, TN> s;
  __shared__ TileMap<TM, TN> m;
  // The base tables are indexed per contribution and per output job.  They
  // are copied from the kernel arguments to LDS with constant indices only:
  // an argument indexed by a run-time value (or passed by address) is first
  // copied to every lane's private scratch memory.
  __shared__ Bases sb, so;
  // block-cyclic XCD remap of the products stage: workgroup b runs on XCD
  // b % 8; each XCD takes chunks of C consecutive tiles in turn, so
  // neighbouring tiles (sharing an operand tile) run on one L2 while the
  // chunks stay balanced.  (The accumulation stage measured faster without.)
  constexpr int C = 32;
  const int G = int(gridDim.x), bb = int(blockIdx.x), full = (G / (8 * C)) * (8 * C);
  int bx = bb;
  if (ROLE == 0 && bb < full) {
    const int x = bb & 7, q = bb >> 3;
    bx = ((q / C) * 8 + x) * C + (q % C);
  }
  if (!ib && threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kMaxBases; ++k) {
      sb.p[k] = bs.p[k];
      sb.stride[k] = bs.stride[k];
      so.p[k] = bout.p[k];
      so.stride[k] = bout.stride[k];
    }
  }
  // (the barrier after the tile maps orders these writes before any read)
  if constexpr (Persist<MODE>::on) {
    for (int ti = bx; ti < ntiles; ti += gridDim.x) {
      __syncthreads();  // the previous tile is done with the maps and bases
      do_tile<MODE, TM, TN>(ti, tiles, jobs, con, gather, segs, nslots, partial, fold, batch, out_f64, s, m, sb,
                            so, ib);
    }
  } else {
    do_tile<MODE, TM, TN>(bx, tiles, jobs, con, gather, segs, nslots, partial, fold, batch, out_f64, s, m, sb, so,
                          ib);
  }
}

// Sum the partial tiles of each reduction item in segment order and write
// the tile to its output block.
template <class PT, int TM, int TN>
__global__ __launch_bounds__(NTH) void reduce_partials_kernel(const GRed* __restrict__ red,
                                                              const GJob* __restrict__ jobs,
                                                              const PT* __restrict__ partial, int nslots, Bases bout0,
                                                              int fold, int batch, int out_f64,
                                                              const Bases* __restrict__ ib) {
  __shared__ TileMap<TM, TN> m;
  const GRed r = red[blockIdx.x];
  const GJob J = jobs[r.job];
  const Bases& bout = ib ? ib[J.inst] : bout0;
  const int tid = threadIdx.x;
  tile_maps<TM, TN>(m, J, r.tm, r.tn, fold, batch, tid, nullptr);
  __syncthreads();
  const long entry = fold == 0 ? long(blockIdx.y) : 0;
  const PT* P = partial + (entry * nslots + r.slot0) * long(TM * TN);
  for (int e = tid; e < TM * TN; e += NTH) {
    const int i = e / TN, j = e % TN;
    if (m.ri[i] < 0 || m.cj[j] < 0) continue;
    double sum = 0;
    for (int q = 0; q < r.nseg; ++q) sum += double(P[long(q) * TM * TN + e]);
    if (out_f64) put_out<double>(bout, J, m, fold, i, j, sum);
    else put_out<float>(bout, J, m, fold, i, j, sum);
  }
}

__global__ void diag_add_f32_kernel(const DiagAdd* __restrict__ d, Bases bs0, const Bases* __restrict__ ib) {
  const DiagAdd x = d[blockIdx.x];
  const Bases& bs = ib ? ib[x.inst] : bs0;
  float* o = reinterpret_cast<float*>(bs.p[x.base]) + x.off + long(blockIdx.y) * bs.stride[x.base];
  for (int i = threadIdx.x; i < x.dim; i += blockDim.x) o[long(i) * (x.dim + 1)] += float(x.c);
}

__global__ void convert_f64_f32_kernel(const double* __restrict__ in, float* __restrict__ out, long n) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x)
    out[e] = float(in[e]);
}

__global__ void convert_list_kernel(const ConvJob* __restrict__ jobs) {
  const ConvJob j = jobs[blockIdx.y];
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < j.n; e += long(gridDim.x) * blockDim.x)
    j.out[e] = float(j.in[e]);
}

template <int MODE, int TM, int TN>
void launch_shape(int role, dim3 grid, hipStream_t s, const GTile* tiles, int ntiles, const GJob* jobs,
                  const GContrib* con, const int* gather, const GSeg* segs, int nslots, void* partial, const Bases& b, const Bases& bout, int fold, int batch,
                  int of, const Bases* ib) {
  typedef typename Cfg<MODE>::T T;
  T* P = static_cast<T*>(partial);
  constexpr int NT = Geo<TM, TN>::NT;
  if (role == 0)
    hipLaunchKernelGGL((ggemm_mfma_kernel<MODE, 0, TM, TN>), grid, dim3(NT), 0, s, tiles, ntiles, jobs, con,
                       gather, segs, nslots, P, b, bout, fold, batch, of, ib);
  else
    hipLaunchKernelGGL((ggemm_mfma_kernel<MODE, 1, TM, TN>), grid, dim3(NT), 0, s, tiles, ntiles, jobs, con,
                       gather, segs, nslots, P, b, bout, fold, batch, of, ib);
}

template <int MODE>
void launch_mode(int shape, int role, dim3 grid, hipStream_t s, const GTile* tiles, int ntiles, const GJob* jobs,
                 const GContrib* con, const int* gather, const GSeg* segs, int nslots, void* partial, const Bases& b, const Bases& bout,
                 int fold, int batch, int of, const Bases* ib) {
  if (MODE != 0 && shape == TILE_128x128)
    launch_shape<MODE, 128, 128>(role, grid, s, tiles, ntiles, jobs, con, gather, segs, nslots, partial, b, bout,
                                 fold, batch, of, ib);
  else if (shape == TILE_128x64)
    launch_shape<MODE, 128, 64>(role, grid, s, tiles, ntiles, jobs, con, gather, segs, nslots, partial, b, bout, fold,
                                batch, of, ib);
  else if (shape == TILE_64x128)
    launch_shape<MODE, 64, 128>(role, grid, s, tiles, ntiles, jobs, con, gather, segs, nslots, partial, b, bout, fold,
                                batch, of, ib);
  else
    launch_shape<MODE, 64, 64>(role, grid, s, tiles, ntiles, jobs, con, gather, segs, nslots, partial, b, bout, fold,
                               batch, of, ib);
}

template <class PT, int TM, int TN>
void launch_reduce(dim3 grid, hipStream_t s, const GRed* red, const GJob* jobs, const void* partial, int nslots,
                   const Bases& bout, int fold, int batch, int of, const Bases* ib) {
  hipLaunchKernelGGL((reduce_partials_kernel<PT, TM, TN>), grid, dim3(NTH), 0, s, red, jobs,
                     static_cast<const PT*>(partial), nslots, bout, fold, batch, of, ib);
}

}  // namespace

int tile_rows(int shape) { return shape == TILE_128x64 || shape == TILE_128x128 ? 128 : 64; }
int tile_cols(int shape) { return shape == TILE_64x128 || shape == TILE_128x128 ? 128 : 64; }

void launch_grouped_gemm(int prec, bool out_f64, int role, int shape, const GTile* tiles, int ntiles,
                         const GJob* jobs, const GContrib* con, const int* gather, const GSeg* segs, int nslots,
                         void* partial, const Bases& b, const Bases& bout, int fold, int batch, hipStream_t s,
                         const Bases* ib) {
  if (ntiles <= 0 || batch <= 0) return;
  // FP64 runs persistent workgroups (at most 16 per CU of the 256, a few
  // rounds of the resident capacity); the others one workgroup per tile
  const int per = fold == 0 ? batch : 1;
  const int cap = 4096 * 16 / per > 0 ? 4096 * 16 / per : 1;
  const int gx = (prec == 0 && ntiles > cap) ? cap : ntiles;
  const dim3 grid(gx, per);
  const int of = out_f64 ? 1 : 0;
  if (prec == 0)
    launch_mode<0>(shape, role, grid, s, tiles, ntiles, jobs, con, gather, segs, nslots, partial, b, bout, fold, batch,
                   1, ib);
  else if (prec == 1)
    launch_mode<1>(shape, role, grid, s, tiles, ntiles, jobs, con, gather, segs, nslots, partial, b, bout, fold, batch,
                   of, ib);
  else
    launch_mode<2>(shape, role, grid, s, tiles, ntiles, jobs, con, gather, segs, nslots, partial, b, bout, fold, batch,
                   of, ib);
}

void launch_reduce_partials(int prec, bool out_f64, int shape, const GRed* red, int nred, const GJob* jobs,
                            int nslots, const void* partial, const Bases& bout, int fold, int batch, hipStream_t s,
                            const Bases* ib) {
  if (nred <= 0 || batch <= 0) return;
  const dim3 grid(nred, fold == 0 ? batch : 1);
  const int of = (prec == 0 || out_f64) ? 1 : 0;
  if (prec == 0) {
    if (shape == TILE_128x64) launch_reduce<double, 128, 64>(grid, s, red, jobs, partial, nslots, bout, fold, batch, 1, ib);
    else if (shape == TILE_64x128)
      launch_reduce<double, 64, 128>(grid, s, red, jobs, partial, nslots, bout, fold, batch, 1, ib);
    else launch_reduce<double, 64, 64>(grid, s, red, jobs, partial, nslots, bout, fold, batch, 1, ib);
  } else {
    if (shape == TILE_128x128)
      launch_reduce<float, 128, 128>(grid, s, red, jobs, partial, nslots, bout, fold, batch, of, ib);
    else if (shape == TILE_128x64) launch_reduce<float, 128, 64>(grid, s, red, jobs, partial, nslots, bout, fold, batch, of, ib);
    else if (shape == TILE_64x128)
      launch_reduce<float, 64, 128>(grid, s, red, jobs, partial, nslots, bout, fold, batch, of, ib);
    else launch_reduce<float, 64, 64>(grid, s, red, jobs, partial, nslots, bout, fold, batch, of, ib);
  }
}

void launch_diag_add_f32(const DiagAdd* d, int n, const Bases& b, int batch, hipStream_t s, const Bases* ib) {
  if (n <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(diag_add_f32_kernel, dim3(n, batch), dim3(256), 0, s, d, b, ib);
}

void launch_convert_list(const ConvJob* jobs, int njobs, long max_n, hipStream_t s) {
  if (njobs <= 0 || max_n <= 0) return;
  long blocks = (max_n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(convert_list_kernel, dim3(unsigned(blocks), njobs), dim3(256), 0, s, jobs);
}

void launch_convert_f64_f32(const double* in, float* out, long n, hipStream_t s) {
  if (n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(convert_f64_f32_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, in, out, n);
}

}  // namespace dmrg
