// Context, operator sets and the contraction planners (host side).
#pragma once
#include <functional>
#include <map>
#include <thread>
#include <mutex>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "qc_mpo.hpp"

namespace dmrg {

class Ctx;

// Owned device allocation (through the context's allocator).
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Ctx* owner = nullptr;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept;
  ~DBuf() { release(); }
  void alloc(Ctx* c, size_t nbytes);
  void ensure(Ctx* c, size_t nbytes);  // grow-only
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Workspace slots of a sigma: dressed operators, stage-1 products, FP32 copy
// of the input vectors, partial tiles of split contribution lists.
enum : int { WS_DRESS = 0, WS_T = 1, WS_C32 = 2, WS_PART = 3, WS_NSLOTS = 4 };
struct WsNeed {
  size_t bytes[WS_NSLOTS] = {0, 0, 0, 0};
};

// Statically allocated device scratch of the no-allocation sigma
// (noalloc.hip): its size and this device's address of it (the device must
// be current; looked up once per device).
size_t scratch_bytes();
void* scratch_address(int device);

// Base slots of the work lists (see kernels.hpp).
enum : int {
  B_CIN = 0, B_SOUT = 1, B_T = 2, B_LOPS = 3, B_ROPS = 4, B_DRESS = 5,
  B_ABRA = 6, B_AKET = 7, B_SRC = 8, B_DST = 9, B_BLK = 10, B_AUX = 11
};

enum RefKind : int { REF_OP = 0, REF_IDENTITY = 1, REF_ZERO = 2 };

// Reference to an operator (or the identity / zero) inside some base.
struct ORef {
  long off = 0;
  const OpLayout* lay = nullptr;
  int kind = REF_IDENTITY;
  int base = -1;
  bool op() const { return kind == REF_OP; }
};

// Operators of one block at one bond for every channel w: side 0 the
// left-block operators Lop_b[w], side 1 the right-block operators Rop_b[w].
// A first-order set (bra zeroth order, ket first order) holds nvec copies and
// its identity channel is zero.
struct OpSet {
  int bond = -1, side = 0, nvec = 1;
  bool first_order = false;
  std::vector<int> kind;  // per channel: REF_OP / REF_IDENTITY / REF_ZERO
  std::vector<long> off;
  std::vector<const OpLayout*> lay;
  long per_vec = 0;
  bool f32 = false;        // data held in FP32 (first-order sets of an FP32 / BF16x3 run)
  DBuf data;
  DBuf data32;             // FP32 copy of FP64 data for the lower-precision contractions
  bool f32_valid = false;
  bool valid() const { return bond >= 0; }
  ORef ref(int w, int base) const {
    ORef r;
    r.kind = kind[w];
    r.base = base;
    r.off = off[w];
    r.lay = lay[w];
    return r;
  }
  double* ptr() const { return data.as<double>(); }
  size_t bytes() const { return data.bytes; }
};

// Device-resident grouped-GEMM list.
struct GemmPlan {
  DBuf tiles, jobs, con, gat;  // gat: gather entries of jobs with a gathered operand
  int ntiles = 0;
  double flops = 0;  // per batch entry
  // host copies for batch folding: job shapes and the bases each operand
  // role reads or writes (bit per base slot)
  std::vector<std::pair<int, int>> shapes;
  std::vector<std::pair<int, int>> ranges;  // contribution range per job
  std::vector<int> con_k;                   // inner length per contribution
  unsigned mask_a = 0, mask_b = 0, mask_c = 0;
  long ncon = 0, kchunks = 0, kchunks_max = 0;  // plan statistics (K-chunks of 32)
  // algorithmic operand elements: distinct A blocks, distinct B blocks, and
  // output elements (each read once, outputs written once) per batch entry
  double elems_a = 0, elems_b = 0, elems_c = 0;
  // launch lists per (fold, batch): tiles with split contribution lists and
  // the reductions of their partial sums
  struct FoldTiles {
    DBuf tiles, segs, red;
    int ntiles = 0, nred = 0, nslots = 0, shape = 0;
  };
  mutable std::map<std::tuple<int, int, int>, FoldTiles> fold_tiles;  // (fold, batch, shape or -1)
  // want: a tile shape, or -1 for the planner's choice
  const FoldTiles& fold_lists(Ctx& x, int fold, int batch, int want = -1) const;
  // prec: DMRG_FP64 (FP64 MFMA), DMRG_FP32 or DMRG_BF16X3 (FP32 operands);
  // outputs go through bout when given (FP64 outputs of a lower-precision run)
  // role 1 marks the accumulation stage (the dominant kernel of a sigma):
  // its main kernel is bracketed by the timing events of a timed sigma
  void launch(Ctx& x, const Bases& b, int batch, int prec = 0, bool out_f64 = true,
              const Bases* bout = nullptr, int role = 0) const;
};

void build_gemm_plan(Ctx& x, GemmPlan& P, std::vector<GJob>& jobs, std::vector<std::vector<GContrib>>& per,
                     const std::vector<int>& gather = {});

struct LinCombPlan {
  DBuf t, s, d, g, u, coef, coef32;  // coef32: the coefficients rounded to FP32
  int nt = 0, nd = 0, ng = 0;
  long max_size = 0;
  double elems = 0, reads = 0;  // plan statistics: target elements, source element reads
  void launch(Ctx& x, const Bases& b, int batch, int prec = 0) const;
};

// Host-side builder of a two-stage contraction (stage 1 writes workspace
// blocks T, stage 2 consumes them), chunked so that T fits a budget.
struct TwoStageBuilder {
  // merge: 0 alone; 1 rows may be stacked with other items sharing op(B)
  // (gathered A rows); 2 columns may be placed side by side with other
  // items sharing op(A) (gathered B columns)
  struct T1 { long elems; GJob job; GContrib con; int merge; };
  // t_is_a: the stage-1 product is operand A of the stage-2 contribution
  // (else operand B)
  struct S2 { int t1; long offC; int baseC, ldc, m, n; GContrib con; bool t_is_a; };
  std::vector<T1> t1;
  std::map<std::tuple<int, long, int>, int> t1_of;  // (base, offset, block) -> item
  std::vector<S2> s2;
  std::vector<std::tuple<long, int, int, int, int>> outputs;  // all outputs (overwrite mode)
};

struct TwoStagePlan {
  std::vector<std::pair<GemmPlan, GemmPlan>> chunks;
  long t_per_vec = 0;
  double flops1 = 0, flops2 = 0;  // per batch entry
};

// Cached plan of one renormalization or sigma variant.
struct ContractionPlan {
  LinCombPlan form;   // dressed operators
  TwoStagePlan main;  // T and outputs
  LinCombPlan post;   // building blocks -> targets
  long dressed_per_vec = 0, blocks_per_vec = 0;
  bool dress_left = true;
  bool bra_first = false;  // renormalization: stage 1 forms A_bra^T X (shared by all kets)
  bool left_first = false;  // sigma: stage 1 forms X C (shared when only Z is batched)
};

struct DiagPlan {
  LinCombPlan form;
  DBuf jobs, terms;
  int njobs = 0;
  long dressed_per_vec = 0;
};

struct SiteTensors {
  DBuf L, R, C;  // device FP64, flat one-site layout
};

// Per-site GEMM plans of the gauge transforms and projections of first-order
// tensors (Sec. II B, eqs. gauge_fwd, gauge_bwd, left1st, right1st; Sec. III
// B, eq. cwfn1st): bond matrices A^T B contracted over (l, n) or over (n, r),
// left / right multiplication of a site tensor by a bond matrix, and scaling
// by Lambda or its inverse.  Bond matrices are block diagonal over the bond's
// sectors (dense m_q x m_q blocks, consecutive).  Built once per MPS; every
// call is batched over `batch` tensors with the given strides.
class GaugeKit {
 public:
  explicit GaugeKit(Ctx& x);
  std::vector<long> size;                 // elements of the one-site tensor per site
  std::vector<std::vector<long>> bm_off;  // per bond: offset of each sector block
  std::vector<long> bm_size;              // per bond: elements of one bond matrix
  long max_size = 1, max_bm = 1;
  // out[bond i+1] = sum over (a, n) of A(a,n,c)^T B(a,n,c)
  void lt(int i, const double* A, long sa, const double* B, long sb, double* out, int batch);
  // out[bond i] = sum over (n, c) of A(a,n,c) B(a,n,c)^T
  void rt(int i, const double* A, long sa, const double* B, long sb, double* out, int batch);
  // Out(a,n,c) (+|-)= M[a] A(a,n,c)
  void lmul(int i, bool add, const double* M, long sm, const double* A, long sa, double* out, int batch);
  // Out(a,n,c) (+|-)= A(a,n,c) M[c]
  void rmul(int i, bool add, const double* A, long sa, const double* M, long sm, double* out, int batch);
  // rows (by Lambda of bond i) or columns (Lambda of bond i+1), or their inverses
  void scale(int i, bool rows, bool inverse, double* data, int batch);
  // Q^L projection out = A - L_i (L_i^T A) and Q^R projection
  // out = A - (A R_i^T) R_i; bm must hold batch bond matrices of bond i+1
  // (left) or bond i (right); out may equal A
  void q_left(int i, const double* A, double* out, double* bm, int batch);
  void q_right(int i, const double* A, double* out, double* bm, int batch);

 private:
  Ctx& x_;
  struct SiteOps {
    GemmPlan lt, rt, lmul_add, lmul_sub, rmul_sub, rmul_add;
    DBuf scale_rows, scale_cols;  // BlockScale lists
    int nrows = 0, ncols = 0;
  };
  std::vector<SiteOps> sp_;
};

// First-order block operators built by dmrg_renormalize with order 1
// (Sec. III B eq. lopr1st, Sec. III D eq. ropr1st), one chain per side: the
// set at `bond` for nvec first-order tensors, ping-ponged between two
// buffers as the chain grows by one site per call.
struct FirstOrderChain {
  OpSet set[2];
  int cur = 0, bond = -1, nvec = 0, prec = -1;
  const OpSet& at() const { return set[cur]; }
  void reset() {
    bond = -1;
    nvec = 0;
    prec = -1;
    cur = 0;
    for (auto& s : set) s = OpSet();
  }
};

// Appends one JSON object as a line to the file named by DMRG_LOG_JSONL, if
// set (per-sweep / per-iteration metrics of the drivers); thread-safe.
void log_jsonl(const std::string& json_object);

// Host copy of an MPS in the import / export format.
struct MpsHostCopy {
  std::vector<int> nsec, sec;
  std::vector<double> L, R, C, lam;
};

class SigmaGroup;

class Ctx {
  friend class SigmaGroup;

 public:
  Ctx(int L, int na, int nb, const double* h, const double* eri, double ecore, int device, void* stream,
      const dmrg_allocator* alloc);
  // bumped whenever the MPS or the zeroth-order operator pools change
  // (grouped launches hold pointers into them)
  unsigned long generation = 0;
  ~Ctx();

  int L, Na, Nb;
  int device;
  hipStream_t stream = nullptr;
  dmrg_allocator allocator{};
  std::string err;
  std::unique_ptr<QCHamiltonian> H;
  long t_budget_per_vec;  // workspace elements per batch entry
  bool fp64_mfma = true;   // FP64 grouped GEMM on matrix cores (else FMA kernel)
  // tile shape per (precision, stage, fold); -1 = the planner's choice
  int tile_policy[3][2][3];
  // time the sigma at `site` for nvec vectors under each pair of stage-1 /
  // stage-2 tile shapes and keep the fastest for precision prec
  void autotune(int site, int nvec, int prec, int* shapes, double* best_ms);

  // MPS
  bool have_mps = false;
  std::vector<Bond> bonds;
  std::vector<std::vector<std::vector<double>>> lam;  // [bond][sector] host
  std::vector<SiteTensors> site;
  std::vector<DBuf> lam_dev, laminv_dev;  // per bond, flat over sectors
  const SiteLayout& layout(int i, int width);
  const OpLayout* op_layout(int bond, int dna, int dnb);
  long bond_offset(int b, int sector) const;  // offset of a sector in the flat bond vector

  // zeroth-order operators
  std::vector<OpSet> left, right;  // left[b] = Lop_b, right[b] = Rop_b
  int ops_prec = -1;

  // workspaces
  DBuf ws_T, ws_dress, ws_blk, ws_aux, ws_c32, ws_part, ws_a32;
  DBuf ws_fo, ws_tda;  // projected first-order tensors; partial TDA sigmas
  // free every grow-only workspace (after a sweep run, whose batched
  // contractions grow them far beyond what a single sigma needs)
  void release_workspaces();

  dmrg_stats stats{};

  void* dev_alloc(size_t bytes);
  void dev_free(void* p);
  void require_gpu() const;
  void sync();

  void import_mps(const int* nsec, const int* sectors, const double* Ld, const double* Rd, const double* Cd,
                  const double* lam);
  void export_mps(int* nsec_out, int* sectors_out, double* Ld, double* Rd, double* Cd, double* lam_out,
                  size_t* sizes);
  void upload_lambda();
  void build_ops(int prec);
  // reuse: keep the set's buffer when it is large enough (no reallocation)
  void alloc_opset(OpSet& S, int bond, int side, int nvec, bool first_order, bool reuse = false, bool f32 = false);
  long opset_size(int bond, int side);  // elements per vector of the set at (bond, side)

  // Renormalization across site i into dst (left: bond i -> i+1; right:
  // bond i+1 -> i).  bra tensor Abra with batch stride abra_stride and ket
  // tensor Aket with batch stride aket_stride (0 = shared; at most one of the
  // two tensors, and then not the source set, is batched), src / dst operator
  // sets (batched sets carry their own stride).  accumulate: add into dst
  // instead of overwriting it.
  void renorm(int dir, int i, const double* Abra, const double* Aket, long aket_stride, const OpSet& src,
              OpSet& dst, bool accumulate, int batch, int prec = 0, long abra_stride = 0);
  // sigma = H_eff C with the left set X and the right set Z on the dot
  // (i, width); C has batch stride cstride (0 = shared), outputs have stride
  // sstride; batch = number of outputs.
  void sigma_general(int i, int width, const OpSet& X, const OpSet& Z, const double* C, long cstride, double* S,
                     long sstride, int batch, int prec = 0);
  void sigma(int i, int width, int nvec, const double* Cin, double* Sout, int prec = 0);
  // dmrg_renormalize with order 1: grow the first-order chain of side dir by
  // site i with the nvec first-order tensors A1 (device FP64, flat layout)
  void renorm_first(int i, int dir, int nvec, const double* A1, int prec);
  // dmrg_sigma with a TDA kind (DMRG_SIGMA_TDA_FULL / TDA_DH_LEFT) at site i
  void sigma_tda(int i, int kind, int nvec, const double* Cin, double* Sout, int prec);
  FirstOrderChain fo_chain[2];  // [0]: left sets, [1]: right sets
  // reduced matrices H_R, S_R of the last dmrg_tda_roots iteration (host,
  // row-major l x l)
  std::vector<double> tda_hr, tda_sr;
  int tda_l = 0;
  // dmrg_sigma_noalloc: the zeroth-order sigma with its workspaces carved from
  // the static scratch; any device allocation inside it is an error
  void sigma_noalloc(int i, int width, int nvec, const double* Cin, double* Sout, int prec);
  // device memory of a workspace slot: the owned buffer grown on demand, or in
  // a no-allocation call the slot's fixed region of the scratch
  void* workspace(int slot, DBuf& buf, size_t bytes);
  WsNeed ws_need_;  // peak bytes per slot since the last reset
  std::map<std::tuple<int, int, int, int>, WsNeed> sigma_need_;  // (site, width, nvec, prec)
  void* scratch_ = nullptr;
  bool no_alloc_ = false;
  size_t carve_off_[WS_NSLOTS] = {0, 0, 0, 0}, carve_len_[WS_NSLOTS] = {0, 0, 0, 0};
  GaugeKit& gauge_kit();
  void drop_gauge_kit();
  // record device time of f() (and of the dominant launches inside it) into
  // stats.sigma_ms / sigma_main_ms / sigma_main_launches
  template <class F> void timed_sigma(F&& f);
  void ensure_f32(const OpSet& S);
  // FP32 operands of a set: its own data when held in FP32, else the
  // converted copy
  float* f32_data(const OpSet& S);
  // events bracketing the dominant (stage-2) launches of a timed sigma
  void mark_main(bool begin);
  bool timing_main_ = false;
  std::vector<hipEvent_t> main_events_;
  int main_events_used_ = 0;
  void diag(int i, int width, double* out);
  void tda_roots(int nroots, const dmrg_davidson_params& p, double* omega, double* etot, double* resid2,
                 int* iters, bool* converged);
  void rpa_roots(int nroots, const dmrg_davidson_params& p, double* omega, double* etot, double* resid2,
                 int* iters, bool* converged);
  void response(const double* v, double omega, const dmrg_davidson_params& p, double* chi, double* resid2,
                int* iters, bool* converged);
  void export_host(MpsHostCopy& m);
  void onebody_rhs(const double* v, const MpsHostCopy& m, double* rhs, const std::vector<long>& off);
  // DMRG-TDA roots and their one-particle transition densities
  void tda_transition(int nroots, const dmrg_davidson_params& p, double* omega, double* etot, double* resid2,
                      int* iters, bool* converged, double* gamma);
  // all plans of the TDA sweeps, built on the plan threads
  void prebuild_tda_plans();
  // ground state by two-site sweeps (ground.cpp); returns <Psi|H|Psi>
  void sweep_ground(const dmrg_sweep_params& p, double* energy, double* discarded, bool* converged);
  // replace the sectors of bond b (and its Schmidt values); drops every
  // cached layout, plan and operator set that depends on bond b
  void set_bond(int b, Bond nb, std::vector<std::vector<double>> lam_b);
  void invalidate_bond(int b);
  void upload_lambda_bond(int b);

 private:
  std::unique_ptr<GaugeKit> kit_;
  std::map<std::pair<int, int>, std::unique_ptr<SiteLayout>> layouts_;
  std::map<std::tuple<int, int, int>, std::unique_ptr<OpLayout>> op_layouts_;
  std::mutex op_layout_mu_;  // op_layout() is called from the plan threads
  std::map<std::tuple<int, int, int, int>, std::unique_ptr<ContractionPlan>> renorm_plans_;
  std::map<std::tuple<int, int, int, int>, std::unique_ptr<ContractionPlan>> sigma_plans_;
  std::map<std::pair<int, int>, std::unique_ptr<DiagPlan>> diag_plans_;
  ContractionPlan& renorm_plan(int dir, int i, const OpSet& src, const OpSet& dst, bool bra_first);
  std::unique_ptr<ContractionPlan> make_renorm_plan(int dir, int i, const OpSet& src, const OpSet& dst,
                                                   bool bra_first);
  std::unique_ptr<ContractionPlan> make_sigma_plan(int i, int width, const OpSet& X, const OpSet& Z, bool left_first);
  // fn(0 .. n-1) on the plan threads (exceptions rethrown afterwards)
  void parallel_for(int n, const std::function<void(int)>& fn);
  // runs plan builders on the plan threads (results in the order given)
  std::vector<std::unique_ptr<ContractionPlan>> build_parallel(
      const std::vector<std::function<std::unique_ptr<ContractionPlan>()>>& fns);
  // host threads for plan construction: DMRG_PLAN_THREADS, else up to 16
  static int plan_threads() {
    if (const char* e = std::getenv("DMRG_PLAN_THREADS")) return std::max(1, std::atoi(e));
    const unsigned h = std::thread::hardware_concurrency();
    return int(std::min(16u, std::max(1u, h)));
  }
  ContractionPlan& sigma_plan(int i, int width, const OpSet& X, const OpSet& Z, bool left_first = false);
  void clear_plans();
};

}  // namespace dmrg

namespace dmrg {

template <class F>
void Ctx::timed_sigma(F&& f) {
  hipEvent_t e0, e1;
  DMRG_HIP(hipEventCreate(&e0));
  DMRG_HIP(hipEventCreate(&e1));
  main_events_used_ = 0;
  timing_main_ = true;
  DMRG_HIP(hipEventRecord(e0, stream));
  try {
    f();
  } catch (...) {
    timing_main_ = false;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  timing_main_ = false;
  DMRG_HIP(hipEventRecord(e1, stream));
  DMRG_HIP(hipEventSynchronize(e1));
  float ms = 0;
  DMRG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  stats.sigma_ms = ms;
  double main_ms = 0;
  for (int k = 0; k + 1 < main_events_used_; k += 2) {
    float d = 0;
    DMRG_HIP(hipEventElapsedTime(&d, main_events_[k], main_events_[k + 1]));
    main_ms += d;
  }
  stats.sigma_main_ms = main_ms;
  stats.sigma_main_launches = main_events_used_ / 2;
}

}  // namespace dmrg

// Opaque handle of the C-ABI (include/dmrg.h).
struct dmrg_ctx {
  dmrg::Ctx* x;
};
