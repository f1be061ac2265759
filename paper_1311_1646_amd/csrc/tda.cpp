// DMRG-TDA by the sweep Davidson algorithm (Sec. III of the paper, Fig.
// alg:dmrgtda), all data device resident in FP64.
//
// Trial vectors are first-order MPS changes.  A forward sweep (site 0..L-1)
// Ritz-rotates the right-gauge objects of the previous iteration (eq.
// ritzrot2), moves the mixed-canonical centre with eq. gauge_fwd, forms the
// sigma of eq. sigv1 (zeroth-order part, first-order left part, and the
// stored first-order right part), the residual (eq. rnorm), the
// diagonal-preconditioned correction (eq. error) projected by Q^C (eq.
// param), the projected coefficients of eq. cwfn1st, accumulates H_R and S_R
// (eqs. hleft2, sleft2) and builds L^(1) (eq. left1st) and the first-order
// left operators (eq. lopr1st).  The backward sweep brings every trial vector
// to the right gauge (eq. gauge_bwd, eq. right1st), builds the first-order
// right operators (eq. ropr1st) and stores, per site, the first-order right
// part of the sigma contracted with C^(0) (it is linear in the right
// operators, so it is rotated instead of the operators themselves).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <string>

#include "engine.hpp"
#include "rpa_reduced.hpp"

namespace dmrg {

namespace {

template <class T>
void upload_vec(Ctx& x, DBuf& buf, const std::vector<T>& v) {
  buf.alloc(&x, std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty()) DMRG_HIP(hipMemcpy(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// deterministic normal deviates (splitmix64 + Box-Muller)
struct HostRng {
  uint64_t s;
  explicit HostRng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ULL + 12345) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return (double(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u = uniform(), v = uniform();
    return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
  }
};


}  // namespace

GaugeKit::GaugeKit(Ctx& x) : x_(x) {
  const int L = x.L;
  size.resize(L);
  for (int i = 0; i < L; ++i) {
    size[i] = long(x.layout(i, 1).size);
    max_size = std::max(max_size, size[i]);
  }
  bm_off.resize(L + 1);
  bm_size.assign(L + 1, 0);
  for (int b = 0; b <= L; ++b) {
    bm_off[b].resize(x.bonds[b].q.size());
    long o = 0;
    for (size_t s = 0; s < x.bonds[b].q.size(); ++s) {
      bm_off[b][s] = o;
      o += long(x.bonds[b].dim[s]) * x.bonds[b].dim[s];
    }
    bm_size[b] = o;
    max_bm = std::max(max_bm, o);
  }
  sp_.resize(L);
  for (int i = 0; i < L; ++i) {
    const SiteLayout& S = x.layout(i, 1);
    SiteOps& so = sp_[i];
    // lt: out[c] (bond i+1) = sum_{(a,n)->c} A(a,n,c)^T B(a,n,c)
    {
      std::vector<GJob> jobs;
      std::vector<std::vector<GContrib>> per;
      std::map<int, int> jo;
      for (auto& b : S.blk) {
        auto it = jo.find(b.c);
        if (it == jo.end()) {
          GJob j{};
          j.offC = bm_off[i + 1][b.c];
          j.baseC = B_SOUT;
          j.ldc = b.cols;
          j.m = b.cols;
          j.n = b.cols;
          jobs.push_back(j);
          per.emplace_back();
          it = jo.emplace(b.c, int(jobs.size()) - 1).first;
        }
        per[it->second].push_back({long(b.off), long(b.off), b.cols, b.cols, b.rows, GC_TRANS_A, B_ABRA, B_AKET, 1.0});
      }
      build_gemm_plan(x, so.lt, jobs, per);
    }
    // rt: out[a] (bond i) = sum_{(n,c)} A(a,n,c) B(a,n,c)^T
    {
      std::vector<GJob> jobs;
      std::vector<std::vector<GContrib>> per;
      std::map<int, int> jo;
      for (auto& b : S.blk) {
        auto it = jo.find(b.a);
        if (it == jo.end()) {
          GJob j{};
          j.offC = bm_off[i][b.a];
          j.baseC = B_SOUT;
          j.ldc = b.rows;
          j.m = b.rows;
          j.n = b.rows;
          jobs.push_back(j);
          per.emplace_back();
          it = jo.emplace(b.a, int(jobs.size()) - 1).first;
        }
        per[it->second].push_back({long(b.off), long(b.off), b.cols, b.cols, b.cols, GC_TRANS_B, B_ABRA, B_AKET, 1.0});
      }
      build_gemm_plan(x, so.rt, jobs, per);
    }
    // lmul: Out(a,n,c) +-= M[a] A(a,n,c)
    for (int add = 0; add < 2; ++add) {
      std::vector<GJob> jobs;
      std::vector<std::vector<GContrib>> per;
      for (auto& b : S.blk) {
        GJob j{};
        j.offC = long(b.off);
        j.baseC = B_SOUT;
        j.ldc = b.cols;
        j.m = b.rows;
        j.n = b.cols;
        j.flags = GJ_ACCUMULATE;
        jobs.push_back(j);
        per.push_back({{bm_off[i][b.a], long(b.off), b.rows, b.cols, b.rows, 0, B_AUX, B_AKET, add ? 1.0 : -1.0}});
      }
      build_gemm_plan(x, add ? so.lmul_add : so.lmul_sub, jobs, per);
    }
    // rmul: Out(a,n,c) +-= A(a,n,c) M[c]
    for (int add = 0; add < 2; ++add) {
      std::vector<GJob> jobs;
      std::vector<std::vector<GContrib>> per;
      for (auto& b : S.blk) {
        GJob j{};
        j.offC = long(b.off);
        j.baseC = B_SOUT;
        j.ldc = b.cols;
        j.m = b.rows;
        j.n = b.cols;
        j.flags = GJ_ACCUMULATE;
        jobs.push_back(j);
        per.push_back({{long(b.off), bm_off[i + 1][b.c], b.cols, b.cols, b.cols, 0, B_AKET, B_AUX,
                        add ? 1.0 : -1.0}});
      }
      build_gemm_plan(x, add ? so.rmul_add : so.rmul_sub, jobs, per);
    }
    std::vector<BlockScale> rows, cols;
    for (auto& b : S.blk) {
      rows.push_back({long(b.off), x.bond_offset(i, b.a), b.rows, b.cols, 1, 0});
      cols.push_back({long(b.off), x.bond_offset(i + 1, b.c), b.rows, b.cols, 0, 0});
    }
    upload_vec(x, so.scale_rows, rows);
    upload_vec(x, so.scale_cols, cols);
    so.nrows = int(rows.size());
    so.ncols = int(cols.size());
  }
}

void GaugeKit::lt(int i, const double* A, long sa, const double* B, long sb, double* out, int batch) {
  Bases b{};
  b.p[B_ABRA] = const_cast<double*>(A);
  b.stride[B_ABRA] = sa;
  b.p[B_AKET] = const_cast<double*>(B);
  b.stride[B_AKET] = sb;
  b.p[B_SOUT] = out;
  b.stride[B_SOUT] = bm_size[i + 1];
  sp_[i].lt.launch(x_, b, batch);
}

void GaugeKit::rt(int i, const double* A, long sa, const double* B, long sb, double* out, int batch) {
  Bases b{};
  b.p[B_ABRA] = const_cast<double*>(A);
  b.stride[B_ABRA] = sa;
  b.p[B_AKET] = const_cast<double*>(B);
  b.stride[B_AKET] = sb;
  b.p[B_SOUT] = out;
  b.stride[B_SOUT] = bm_size[i];
  sp_[i].rt.launch(x_, b, batch);
}

void GaugeKit::lmul(int i, bool add, const double* M, long sm, const double* A, long sa, double* out, int batch) {
  Bases b{};
  b.p[B_AUX] = const_cast<double*>(M);
  b.stride[B_AUX] = sm;
  b.p[B_AKET] = const_cast<double*>(A);
  b.stride[B_AKET] = sa;
  b.p[B_SOUT] = out;
  b.stride[B_SOUT] = size[i];
  (add ? sp_[i].lmul_add : sp_[i].lmul_sub).launch(x_, b, batch);
}

void GaugeKit::rmul(int i, bool add, const double* A, long sa, const double* M, long sm, double* out, int batch) {
  Bases b{};
  b.p[B_AUX] = const_cast<double*>(M);
  b.stride[B_AUX] = sm;
  b.p[B_AKET] = const_cast<double*>(A);
  b.stride[B_AKET] = sa;
  b.p[B_SOUT] = out;
  b.stride[B_SOUT] = size[i];
  (add ? sp_[i].rmul_add : sp_[i].rmul_sub).launch(x_, b, batch);
}

void GaugeKit::scale(int i, bool rows, bool inverse, double* data, int batch) {
  const int bond = rows ? i : i + 1;
  const DBuf& v = inverse ? x_.laminv_dev[bond] : x_.lam_dev[bond];
  const SiteOps& so = sp_[i];
  launch_block_scale_f64(rows ? so.scale_rows.as<BlockScale>() : so.scale_cols.as<BlockScale>(),
                         rows ? so.nrows : so.ncols, v.as<double>(), data, size[i], batch, x_.stream);
  DMRG_HIP(hipGetLastError());
}

void GaugeKit::q_left(int i, const double* A, double* out, double* bm, int batch) {
  const double* Li = x_.site[i].L.as<double>();
  lt(i, Li, 0, A, size[i], bm, batch);
  if (out != A && batch > 0)
    DMRG_HIP(hipMemcpyAsync(out, A, size_t(batch) * size[i] * 8, hipMemcpyDeviceToDevice, x_.stream));
  rmul(i, false, Li, 0, bm, bm_size[i + 1], out, batch);
}

void GaugeKit::q_right(int i, const double* A, double* out, double* bm, int batch) {
  const double* Ri = x_.site[i].R.as<double>();
  rt(i, A, size[i], Ri, 0, bm, batch);
  if (out != A && batch > 0)
    DMRG_HIP(hipMemcpyAsync(out, A, size_t(batch) * size[i] * 8, hipMemcpyDeviceToDevice, x_.stream));
  lmul(i, false, bm, bm_size[i], Ri, 0, out, batch);
}

GaugeKit& Ctx::gauge_kit() {
  require_gpu();
  DMRG_REQUIRE(have_mps, DMRG_ERR_STATE, "no MPS");
  if (!kit_) kit_.reset(new GaugeKit(*this));
  return *kit_;
}

void Ctx::drop_gauge_kit() { kit_.reset(); }

// Device time of the phases of one Davidson iteration, from events recorded
// on the context's stream between the phases (only when the run is verbose):
// the span from one mark to the next is charged to the first mark's phase.
struct PhaseClock {
  enum { SIG1, SIG0, REN11, REN01, VEC, HOST, N };
  hipStream_t s = nullptr;
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> cat;
  int used = 0;
  double acc[N] = {};
  void mark(int c) {
    if (!on) return;
    if (used == int(ev.size())) {
      hipEvent_t e;
      DMRG_HIP(hipEventCreate(&e));
      ev.push_back(e);
      cat.push_back(0);
    }
    cat[used] = c;
    DMRG_HIP(hipEventRecord(ev[used], s));
    ++used;
  }
  // call after the stream has drained past the last mark
  void collect() {
    if (!on) return;
    for (int k = 0; k + 1 < used; ++k) {
      float ms = 0;
      DMRG_HIP(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
      acc[cat[k]] += ms;
    }
    used = 0;
  }
  ~PhaseClock() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// Frequency-dependent linear response (Sec. II B, eqs. realresp, imagresp):
// the first-order wavefunctions of the +omega and -omega components solve
// (H - z_pm) Psi1_pm = -Q V Psi0 in the tangent space with the reference
// removed, z_pm = E0 -+ omega.  rhs[i] = P_i^T V Psi0 is the site-i
// projection of V Psi0 (flat one-site layout, device FP64).
struct ResponseSpec {
  std::vector<const double*> rhs;
  double omega = 0;
};

class TdaRunner {
 public:
  // nroots TDA roots, or (rs != null) the two response vectors of rs, or
  // (rpa) nroots RPA roots, each with a forward and a backward component
  TdaRunner(Ctx& x, int nroots, const dmrg_davidson_params& p, const ResponseSpec* rs = nullptr, bool rpa = false)
      : x_(x), k_(x.gauge_kit()), n_(rs ? 2 : (rpa ? 2 * nroots : nroots)), p_(p), prec_(p.prec) {
    rpa_ = rpa && !rs;
    nr_ = nroots;
    if (rs) {
      resp_ = true;
      rhs_ = rs->rhs;
      omega_ = rs->omega;
      DMRG_REQUIRE(int(rhs_.size()) == x.L, DMRG_ERR_INTERNAL, "response right-hand side per site");
    }
    L_ = x.L;
    const long maxsize = k_.max_size;
    guess_ = p.guess;
    Nmax_ = p.max_space > 0 ? p.max_space : auto_space();
    DMRG_REQUIRE(Nmax_ <= 64, DMRG_ERR_INVALID_ARG, "max_space must be <= 64");
    DMRG_REQUIRE(n_ >= 1 && 2 * n_ <= Nmax_, DMRG_ERR_INVALID_ARG,
                 rpa_ ? "need 1 <= nroots and 4*nroots <= max_space (RPA: an X and a Y residual per root)"
                      : "need 1 <= nroots and 2*nroots <= max_space");
    x.stats.tda_space = Nmax_;
    // per-site storage
    R1_.resize(L_);
    G_.resize(L_);
    Ct_.resize(L_);
    diag_.resize(L_);
    for (int i = 0; i < L_; ++i) {
      R1_[i].alloc(&x, size_t(Nmax_) * k_.size[i] * 8);
      G_[i].alloc(&x, size_t(Nmax_) * k_.size[i] * 8);
      Ct_[i].alloc(&x, size_t(Nmax_) * k_.size[i] * 8);
      diag_[i].alloc(&x, size_t(k_.size[i]) * 8);
    }
    const size_t vs = size_t(Nmax_) * maxsize * 8;
    for (DBuf* b : {&Cm_, &Cprev_, &Cb_, &Sg_, &S0_, &Dl_, &Wk_, &R1r_, &Gr_}) b->alloc(&x, vs);
    bm_.alloc(&x, size_t(Nmax_) * k_.max_bm * 8);
    HR_.alloc(&x, 64 * 64 * 8);
    SR_.alloc(&x, 64 * 64 * 8);
    alpha_.alloc(&x, 64 * 64 * 8);
    w_.alloc(&x, 64 * 8);
    rank_.alloc(&x, 8);
    negw_.alloc(&x, 64 * 8);
    ones_.alloc(&x, 64 * 8);
    zscale_.alloc(&x, 64 * 8);
    tmpd_.alloc(&x, 64 * 64 * 8);
    part_.alloc(&x, size_t(gram_parts(maxsize) + 1) * 64 * 64 * 8);
    if (resp_) {
      bR_.alloc(&x, 64 * 8);
      cres_.alloc(&x, 64 * 2 * 8);
      zsh_.alloc(&x, 64 * 8);
      for (DBuf* b : {&Cx_, &Dx_, &Gx_}) b->alloc(&x, 2 * size_t(maxsize) * 8);
    }
    if (rpa_) {
      // the second-order parts: Gamma^R per site (eq. bmatrix, backward
      // sweep), Gamma^L of the current site, the W half-matrix, and the
      // coefficients of X and Y (and of Y and X) in the rotated basis
      GB_.resize(L_);
      for (int i = 0; i < L_; ++i) GB_[i].alloc(&x, size_t(Nmax_) * k_.size[i] * 8);
      for (DBuf* b : {&GL_, &GBr_, &Cx_, &Dx_, &Gx_, &Xw_}) b->alloc(&x, vs);
      WR_.alloc(&x, 64 * 64 * 8);
      cres_.alloc(&x, 64 * 64 * 8);
      cswap_.alloc(&x, 64 * 64 * 8);
      zsh_.alloc(&x, 64 * 8);
    }
    std::vector<double> one(64, 1.0);
    DMRG_HIP(hipMemcpy(ones_.p, one.data(), 64 * 8, hipMemcpyHostToDevice));
    for (int k = 0; k < 2; ++k) {
      FL_[k].bond = -1;
      FR_[k].bond = -1;
    }
  }

  void run(double* omega, double* etot, double* resid2, int* iters, bool* converged);
  // response mode: <V Psi0 | Psi1_pm> of the last iteration
  double chi(int k) const { return chi_[k]; }
  // after run(): out[nu] = <Psi^nu | v> for the n roots of the last
  // iteration, v given by its site projections P_i^T v (rhs[i]); the roots'
  // left-gauge components are the first n trial vectors of the last forward
  // sweep (S_R-orthonormal Ritz vectors, unit norm)
  void root_overlaps(const std::vector<const double*>& rhs, double* out) {
    for (int i = 0; i < L_; ++i)
      gram(Ct_[i].as<double>(), size(i), n_, rhs[i], size(i), 1, size(i), tmpd_.as<double>(), 1, 1.0, i > 0);
    DMRG_HIP(hipMemcpy(out, tmpd_.p, size_t(n_) * 8, hipMemcpyDeviceToHost));
  }

 private:
  Ctx& x_;
  GaugeKit& k_;
  int n_, L_, Nmax_;
  dmrg_davidson_params p_;
  int prec_;  // contraction precision of sigma and renormalization
  int guess_ = 0;  // initial trial vectors: 0 lowest diagonal at the middle site, 1 random at every site
  std::vector<DBuf> R1_, G_, Ct_, diag_;
  DBuf Cm_, Cprev_, Cb_, Sg_, S0_, Dl_, Wk_, R1r_, Gr_, bm_;
  DBuf HR_, SR_, alpha_, w_, rank_, negw_, ones_, tmpd_, part_, zscale_;
  OpSet FL_[2], FR_[2];
  double E0_ = 0;
  PhaseClock pc_;
  int lcur_last_ = 0;  // size of the reduced matrices of the last forward sweep
  std::vector<double> hw_;  // host copy of Ritz values
  // response mode: right-hand sides, frequency, b_R = <trial | V Psi0>, the
  // coefficients of x_pm in the Ritz basis, the shifts z_pm, and the site
  // pieces of x_pm
  bool resp_ = false;
  std::vector<const double*> rhs_;
  double omega_ = 0, chi_[2] = {0, 0};
  DBuf bR_, cres_, zsh_, Cx_, Dx_, Gx_;
  // RPA mode (Sec. II C eq. dmrgrpa, Sec. III E): nr_ roots; the residual
  // vectors are the n_ = 2 nr_ components X_k, Y_k; first-order operator
  // chains with the first-order tensor on the bra side (FLB_, FRB_) give
  // Gamma^L_i[v] = <U_v n r| H |Psi0> and Gamma^R_i[v] = <l n V_v| H |Psi0>
  // (U_v, V_v the first-order left / right block states of trial vector v)
  bool rpa_ = false;
  int nr_ = 0;
  std::vector<DBuf> GB_;
  DBuf GL_, GBr_, Xw_, WR_, cswap_;
  OpSet FLB_[2], FRB_[2];
  std::vector<double> rpa_omega_;
  // RPA: solve the reduced problem of the l = lcur trial vectors (eq.
  // reducedrpa) and set the basis rotation (alpha_, m columns), the
  // coefficients of the residual vectors and their shifts
  int rpa_step(int lcur, int& m);

  long size(int i) const { return k_.size[i]; }
  void copy(double* dst, const double* src, long n) {
    if (n > 0) DMRG_HIP(hipMemcpyAsync(dst, src, size_t(n) * 8, hipMemcpyDeviceToDevice, x_.stream));
  }
  void gram(const double* A, long lda, int na, const double* B, long ldb, int nb, long n, double* G, int ldg,
            double alpha, bool acc) {
    launch_gram_f64(A, lda, na, B, ldb, nb, n, G, ldg, part_.as<double>(), alpha, acc, x_.stream);
    DMRG_HIP(hipGetLastError());
  }
  void q_c_project(int i, double* z, int nv);  // z -= C0 (C0 . z)
  // response mode, after the small eigenproblem of an iteration: Ritz-basis
  // right-hand side, coefficients of x_pm and chi_pm; reorders the Ritz
  // vectors (alpha, w) by their weight in x_pm so that a restart keeps the
  // important ones
  void response_step(int lcur, int rank, int m, std::vector<double>& w);
  void forward(int m, int lprev, bool init, uint64_t seed, std::vector<double>& r2);
  // size both buffers of a ping-pong pair of first-order sets (side 0 left,
  // 1 right) for the largest bond, so that a sweep allocates once
  void reserve(OpSet* sets, int side, int nvec) {
    long mx = 1;
    for (int b = 0; b <= L_; ++b) mx = std::max(mx, x_.opset_size(b, side));
    const size_t bytes = size_t(mx) * size_t(nvec) * (prec_ != DMRG_FP64 ? 4 : 8);
    for (int k = 0; k < 2; ++k)
      if (sets[k].data.bytes < bytes) sets[k].data.alloc(&x_, bytes);
  }
  void backward(int l);
  // default maximum space: 64 trial vectors, reduced so
  // that the per-vector device memory (two first-order sets of the largest
  // bond and their building blocks, three site vectors per site, nine work
  // vectors) fits in 60% of the free device memory; at least 2n + 2
  int auto_space() {
    long mx = 1;
    for (int b = 0; b <= L_; ++b) mx = std::max({mx, x_.opset_size(b, 0), x_.opset_size(b, 1)});
    long sites = 0;
    for (int i = 0; i < L_; ++i) sites += k_.size[i];
    // sized for FP64 sets whenever the run may end in FP64 polish
    const double esz = (prec_ != DMRG_FP64 && p_.polish != 0) ? 4 : 8;
    const double per = (rpa_ ? 5.0 : 3.0) * double(mx) * esz +
                       8.0 * ((rpa_ ? 4.0 : 3.0) * sites + (rpa_ ? 14.0 : 9.0) * k_.max_size);
    size_t freeb = 0, total = 0;
    int cap = 64;
    if (hipMemGetInfo(&freeb, &total) == hipSuccess) cap = int(std::min(64.0, 0.6 * double(freeb) / per));
    else (void)hipGetLastError();
    const int want = 64;
    return std::max(std::min(want, cap), std::min(64, 2 * n_ + 2));
  }
};

void TdaRunner::response_step(int lcur, int rank, int m, std::vector<double>& w) {
  std::vector<double> al(size_t(lcur) * lcur), br(lcur);
  DMRG_HIP(hipMemcpy(al.data(), alpha_.p, al.size() * 8, hipMemcpyDeviceToHost));
  DMRG_HIP(hipMemcpy(br.data(), bR_.p, br.size() * 8, hipMemcpyDeviceToHost));
  const double z[2] = {E0_ - omega_, E0_ + omega_};
  // b_k = <y_k | V Psi0> for the S_R-orthonormal Ritz vectors y_k (columns of
  // alpha); in that basis (H_R - z S_R) a = -b_R is diagonal:
  // c_k = -b_k / (w_k - z); x_pm = sum_k c_k y_k over all of them
  std::vector<double> b(rank, 0.0), c(size_t(rank) * 2);
  chi_[0] = chi_[1] = 0;
  for (int k = 0; k < rank; ++k) {
    for (int u = 0; u < lcur; ++u) b[k] += al[u + size_t(k) * lcur] * br[u];
    for (int v = 0; v < 2; ++v) {
      c[k + size_t(v) * rank] = -b[k] / (w[k] - z[v]);
      chi_[v] += b[k] * c[k + size_t(v) * rank];
    }
  }
  // Ritz vectors by their weight in x_pm
  std::vector<int> ord(rank);
  for (int k = 0; k < rank; ++k) ord[k] = k;
  std::stable_sort(ord.begin(), ord.end(), [&](int p, int q) {
    return std::abs(c[p]) + std::abs(c[p + rank]) > std::abs(c[q]) + std::abs(c[q + rank]);
  });
  std::vector<double> al2(size_t(lcur) * lcur, 0.0), w2(w), cm(size_t(m) * 2, 0.0);
  if (m >= rank) {
    // the whole Ritz basis is kept: x_pm by their coefficients
    for (int j = 0; j < rank; ++j) {
      const int k = ord[j];
      for (int u = 0; u < lcur; ++u) al2[u + size_t(j) * lcur] = al[u + size_t(k) * lcur];
      w2[j] = w[k];
      for (int v = 0; v < 2; ++v) cm[j + size_t(v) * m] = c[k + size_t(v) * rank];
    }
  } else {
    // restart: the kept space holds x_pm themselves (first columns, so the
    // current solution survives the restart exactly) and the m - 2 (or
    // m - 1 when x_+ = x_-, at omega = 0) Ritz vectors of largest weight
    int col = 0;
    for (int v = 0; v < 2; ++v) {
      if (v == 1 && omega_ == 0.0) break;
      for (int u = 0; u < lcur; ++u) {
        double a = 0;
        for (int k = 0; k < rank; ++k) a += al[u + size_t(k) * lcur] * c[k + size_t(v) * rank];
        al2[u + size_t(col) * lcur] = a;
      }
      cm[col + size_t(v) * m] = 1.0;
      ++col;
    }
    if (omega_ == 0.0) cm[0 + size_t(1) * m] = 1.0;
    for (int j = 0; col < m && j < rank; ++j, ++col) {
      const int k = ord[j];
      for (int u = 0; u < lcur; ++u) al2[u + size_t(col) * lcur] = al[u + size_t(k) * lcur];
      w2[col] = w[k];
    }
  }
  w = w2;
  if (p_.verbose >= 1) {
    double dmin[2] = {1e300, 1e300};
    for (int k = 0; k < rank; ++k)
      for (int v = 0; v < 2; ++v) dmin[v] = std::min(dmin[v], std::abs(w[k] - z[v]));
    std::fprintf(stderr, "[response] rank %d kept %d chi %.12f %.12f  min|w-z| %.3e %.3e\n", rank, m, chi_[0],
                 chi_[1], dmin[0], dmin[1]);
  }
  DMRG_HIP(hipMemcpy(alpha_.p, al2.data(), al2.size() * 8, hipMemcpyHostToDevice));
  DMRG_HIP(hipMemcpy(cres_.p, cm.data(), cm.size() * 8, hipMemcpyHostToDevice));
}

int TdaRunner::rpa_step(int lcur, int& m) {
  const size_t ll = size_t(lcur) * lcur;
  std::vector<double> hr(ll), sr(ll), wh(ll), wr(ll);
  DMRG_HIP(hipMemcpy(hr.data(), HR_.p, ll * 8, hipMemcpyDeviceToHost));
  DMRG_HIP(hipMemcpy(sr.data(), SR_.p, ll * 8, hipMemcpyDeviceToHost));
  DMRG_HIP(hipMemcpy(wh.data(), WR_.p, ll * 8, hipMemcpyDeviceToHost));
  // W_R = W_half + W_half^T (eq. bmatrix, both orders of the pair); the gram
  // layout is W_half[u * lcur + v], symmetric sums need no transpose care
  for (int u = 0; u < lcur; ++u)
    for (int v = 0; v < lcur; ++v) wr[u + size_t(v) * lcur] = wh[u * size_t(lcur) + v] + wh[v * size_t(lcur) + u];
  // H_R and S_R of the gram kernel are [u * lcur + v] too; they are
  // symmetric up to rounding, which the solver symmetrizes
  RpaReduced red;
  const int st = rpa_reduced_solve(lcur, hr.data(), sr.data(), wr.data(), E0_, 1e-10, red);
  DMRG_REQUIRE(st == 0, DMRG_ERR_SINGULAR,
               "RPA stability matrix is not positive definite on the trial space (unstable reference)");
  const int r = red.r;
  DMRG_REQUIRE(r >= nr_, DMRG_ERR_SINGULAR, "trial space lost rank below the number of roots");
  rpa_omega_.assign(red.omega.begin(), red.omega.begin() + nr_);
  // kept basis (coordinates in the orthonormal basis U T, r-vectors): the
  // whole space when it fits, else X' and Y' of the lowest roots,
  // orthonormalized (a restart keeps the current roots exactly)
  std::vector<double> K;  // r x mk, column-major
  int mk = 0;
  if (m >= r) {
    K.assign(size_t(r) * r, 0.0);
    for (int j = 0; j < r; ++j) K[j + size_t(j) * r] = 1.0;
    mk = r;
  } else {
    const int kk = std::min(r, std::max(nr_, m / 2));
    std::vector<double> cand;
    for (int k = 0; k < kk; ++k)
      for (const std::vector<double>* src : {&red.x, &red.y})
        cand.insert(cand.end(), src->begin() + size_t(k) * r, src->begin() + size_t(k + 1) * r);
    const int nc = int(cand.size() / r);
    for (int c = 0; c < nc && mk < m; ++c) {
      std::vector<double> v(cand.begin() + size_t(c) * r, cand.begin() + size_t(c + 1) * r);
      double n0 = 0;
      for (double e : v) n0 += e * e;
      n0 = std::sqrt(n0);
      for (int pass = 0; pass < 2; ++pass)
        for (int j = 0; j < mk; ++j) {
          double d = 0;
          for (int e = 0; e < r; ++e) d += K[e + size_t(j) * r] * v[e];
          for (int e = 0; e < r; ++e) v[e] -= d * K[e + size_t(j) * r];
        }
      double nv = 0;
      for (double e : v) nv += e * e;
      nv = std::sqrt(nv);
      if (nv <= 1e-8 * std::max(n0, 1e-300)) continue;
      for (double& e : v) e /= nv;
      K.insert(K.end(), v.begin(), v.end());
      ++mk;
    }
  }
  m = mk;
  // alpha = T K (lcur x m): the new trial vectors U T K are S-orthonormal
  std::vector<double> al(size_t(lcur) * m, 0.0);
  for (int j = 0; j < m; ++j)
    for (int t = 0; t < r; ++t) {
      const double kv = K[t + size_t(j) * r];
      if (kv == 0.0) continue;
      for (int u = 0; u < lcur; ++u) al[u + size_t(j) * lcur] += red.T[u + size_t(t) * lcur] * kv;
    }
  // residual vectors v < nr_: X_v, v >= nr_: Y_{v - nr_}; coefficients in
  // the new basis K^T X', and the swapped set (Y for the X residuals, X for
  // the Y residuals) that multiplies the W gradients
  std::vector<double> c(size_t(m) * n_, 0.0), cs(size_t(m) * n_, 0.0);
  for (int v = 0; v < nr_; ++v)
    for (int j = 0; j < m; ++j) {
      double dx = 0, dy = 0;
      for (int t = 0; t < r; ++t) {
        dx += K[t + size_t(j) * r] * red.x[t + size_t(v) * r];
        dy += K[t + size_t(j) * r] * red.y[t + size_t(v) * r];
      }
      c[j + size_t(v) * m] = dx;
      c[j + size_t(v + nr_) * m] = dy;
      cs[j + size_t(v) * m] = dy;
      cs[j + size_t(v + nr_) * m] = dx;
    }
  // shifts: X residual (H - (E0 + omega)), Y residual (H - (E0 - omega))
  std::vector<double> z(64, 0.0), nz(64, 0.0);
  for (int v = 0; v < nr_; ++v) {
    z[v] = E0_ + rpa_omega_[v];
    z[v + nr_] = E0_ - rpa_omega_[v];
  }
  for (int v = 0; v < n_; ++v) nz[v] = -z[v];
  if (p_.verbose >= 1) {
    std::fprintf(stderr, "[rpa] rank %d kept %d omega", r, m);
    for (int v = 0; v < nr_; ++v) std::fprintf(stderr, " %.10f", rpa_omega_[v]);
    std::fprintf(stderr, "\n");
  }
  DMRG_HIP(hipMemcpy(alpha_.p, al.data(), al.size() * 8, hipMemcpyHostToDevice));
  DMRG_HIP(hipMemcpy(cres_.p, c.data(), c.size() * 8, hipMemcpyHostToDevice));
  DMRG_HIP(hipMemcpy(cswap_.p, cs.data(), cs.size() * 8, hipMemcpyHostToDevice));
  DMRG_HIP(hipMemcpy(zsh_.p, z.data(), 64 * 8, hipMemcpyHostToDevice));
  DMRG_HIP(hipMemcpy(negw_.p, nz.data(), 64 * 8, hipMemcpyHostToDevice));
  return r;
}

void TdaRunner::q_c_project(int i, double* z, int nv) {
  const double* C0 = x_.site[i].C.as<double>();
  gram(z, size(i), nv, C0, size(i), 1, size(i), tmpd_.as<double>(), 1, -1.0, false);
  launch_axpby_f64(tmpd_.as<double>(), C0, 0, ones_.as<double>(), z, size(i), nv, size(i), x_.stream);
  DMRG_HIP(hipGetLastError());
}

void TdaRunner::forward(int m, int lprev, bool init, uint64_t seed, std::vector<double>& r2) {
  const int l = m + n_;
  r2.assign(n_, 0.0);
  launch_fill_f64(HR_.as<double>(), long(l) * l, 0.0, x_.stream);
  launch_fill_f64(SR_.as<double>(), long(l) * l, 0.0, x_.stream);
  if (resp_) launch_fill_f64(bR_.as<double>(), l, 0.0, x_.stream);
  int cur = 0;
  reserve(FL_, 0, l);
  x_.alloc_opset(FL_[cur], 0, 0, l, true, true, prec_ != DMRG_FP64);
  if (rpa_) {
    reserve(FLB_, 0, l);
    x_.alloc_opset(FLB_[cur], 0, 0, l, true, true, prec_ != DMRG_FP64);
  }
  HostRng rng(seed);
  std::vector<double> tmp;
  for (int i = 0; i < L_; ++i) {
    if (p_.verbose >= 2) std::fprintf(stderr, "[tda] forward site %d (l=%d)\n", i, m + n_);
    const long S = size(i);
    double* Cm = Cm_.as<double>();
    const double* C0 = x_.site[i].C.as<double>();
    // Ritz rotation of the right-gauge objects and gauge shift (eq. gauge_fwd)
    if (m > 0) {
      launch_rotate_f64(R1_[i].as<double>(), S, lprev, alpha_.as<double>(), lprev, m, R1r_.as<double>(), S, S,
                        x_.stream);
      launch_rotate_f64(G_[i].as<double>(), S, lprev, alpha_.as<double>(), lprev, m, Gr_.as<double>(), S, S,
                        x_.stream);
      if (rpa_)
        launch_rotate_f64(GB_[i].as<double>(), S, lprev, alpha_.as<double>(), lprev, m, GBr_.as<double>(), S, S,
                          x_.stream);
      DMRG_HIP(hipGetLastError());
      copy(Cm, R1r_.as<double>(), long(m) * S);
      k_.scale(i, true, false, Cm, m);
      if (i > 0) {
        k_.lt(i - 1, x_.site[i - 1].L.as<double>(), 0, Cprev_.as<double>(), size(i - 1), bm_.as<double>(), m);
        k_.lmul(i, true, bm_.as<double>(), k_.bm_size[i], x_.site[i].R.as<double>(), 0, Cm, m);
      }
    }
    // first-order left part of the sigma for all l vectors (eq. sigv2, first line)
    double* Dl = Dl_.as<double>();
    // the TDA sigma of the middle site (first-order left part for the l
    // trial vectors and zeroth-order part for the n roots) is timed
    const bool timed = !init && i == L_ / 2;
    hipEvent_t te[2] = {nullptr, nullptr};
    double tfl = 0;
    if (timed) {
      DMRG_HIP(hipEventCreate(&te[0]));
      DMRG_HIP(hipEventCreate(&te[1]));
      DMRG_HIP(hipEventRecord(te[0], x_.stream));
    }
    pc_.mark(PhaseClock::SIG1);
    x_.sigma_general(i, 1, FL_[cur], x_.right[i + 1], C0, 0, Dl, S, l, prec_);
    tfl += x_.stats.sigma_flops;
    // RPA: Gamma^L_i[v] = <U_v n r| H |Psi0> (the conjugate first-order
    // superblock operator of eq. bmatrix applied to C^(0))
    if (rpa_) x_.sigma_general(i, 1, FLB_[cur], x_.right[i + 1], C0, 0, GL_.as<double>(), S, l, prec_);
    double* Wk = Wk_.as<double>();
    if (!init) {
      // sigma (eq. sigv1), residual (eq. rnorm), correction (eqs. error, param)
      double* Sg = Sg_.as<double>();
      // the vectors whose residuals are taken: the n lowest Ritz vectors, or
      // in response mode x_pm = sum_k c_k^pm y_k over the m Ritz vectors y_k
      // (their zeroth-order coefficients, first-order left parts and stored
      // right parts rotated alike: the sigma is linear)
      const double* Xc = Cm;
      const double* Xd = Dl;
      const double* Xg = Gr_.as<double>();
      if (resp_ || rpa_) {
        launch_rotate_f64(Cm, S, m, cres_.as<double>(), m, n_, Cx_.as<double>(), S, S, x_.stream);
        launch_rotate_f64(Dl, S, m, cres_.as<double>(), m, n_, Dx_.as<double>(), S, S, x_.stream);
        launch_rotate_f64(Gr_.as<double>(), S, m, cres_.as<double>(), m, n_, Gx_.as<double>(), S, S, x_.stream);
        DMRG_HIP(hipGetLastError());
        Xc = Cx_.as<double>();
        Xd = Dx_.as<double>();
        Xg = Gx_.as<double>();
      }
      if (rpa_) {
        // site-i gradient of W(., v) for the m rotated vectors, Gamma^L_i +
        // Gamma^R_i (the second derivative of the mixed-canonical MPS at
        // site i paired with every first-order piece of v), combined with
        // the swapped coefficients: the X residual takes W Y, the Y
        // residual W X
        launch_axpby_f64(ones_.as<double>(), GBr_.as<double>(), S, ones_.as<double>(), GL_.as<double>(), S, m, S,
                         x_.stream);
        launch_rotate_f64(GL_.as<double>(), S, m, cswap_.as<double>(), m, n_, Xw_.as<double>(), S, S, x_.stream);
        DMRG_HIP(hipGetLastError());
      }
      pc_.mark(PhaseClock::SIG0);
      x_.sigma_general(i, 1, x_.left[i], x_.right[i + 1], Xc, S, Sg, S, n_, prec_);
      pc_.mark(PhaseClock::VEC);
      if (timed) {
        tfl += x_.stats.sigma_flops;
        DMRG_HIP(hipEventRecord(te[1], x_.stream));
        DMRG_HIP(hipEventSynchronize(te[1]));
        float ms = 0;
        DMRG_HIP(hipEventElapsedTime(&ms, te[0], te[1]));
        x_.stats.tda_sigma_ms = ms;
        x_.stats.tda_sigma_flops = tfl;
        (void)hipEventDestroy(te[0]);
        (void)hipEventDestroy(te[1]);
      }
      launch_axpby_f64(ones_.as<double>(), Xd, S, ones_.as<double>(), Sg, S, n_, S, x_.stream);
      launch_axpby_f64(ones_.as<double>(), Xg, S, ones_.as<double>(), Sg, S, n_, S, x_.stream);
      launch_axpby_f64(negw_.as<double>(), Xc, S, ones_.as<double>(), Sg, S, n_, S, x_.stream);
      // response: r = (H - z) x + V Psi0 (eqs. realresp, imagresp)
      if (resp_) launch_axpby_f64(ones_.as<double>(), rhs_[i], 0, ones_.as<double>(), Sg, S, n_, S, x_.stream);
      // RPA: r_X = (H - E0 - omega) X + W Y, r_Y = (H - E0 + omega) Y + W X (eq. dmrgrpa)
      if (rpa_) launch_axpby_f64(ones_.as<double>(), Xw_.as<double>(), S, ones_.as<double>(), Sg, S, n_, S, x_.stream);
      DMRG_HIP(hipGetLastError());
      // residual restricted to the site's tangent directions (orthogonal to
      // C^(0)); for a stationary reference this projection changes nothing
      q_c_project(i, Sg, n_);
      gram(Sg, S, n_, Sg, S, n_, S, tmpd_.as<double>(), n_, 1.0, false);
      tmp.resize(size_t(n_) * n_);
      DMRG_HIP(hipMemcpyAsync(tmp.data(), tmpd_.p, tmp.size() * 8, hipMemcpyDeviceToHost, x_.stream));
      pc_.mark(PhaseClock::HOST);
      x_.sync();
      pc_.mark(PhaseClock::VEC);
      for (int v = 0; v < n_; ++v) r2[v] += tmp[size_t(v) * n_ + v];
      launch_precond_f64(Sg, diag_[i].as<double>(), (resp_ || rpa_) ? zsh_.as<double>() : w_.as<double>(), Wk, n_,
                         S, 1e-8, x_.stream);
      // corrections scaled by 1/|r| of the previous iteration so that new
      // trial vectors keep O(1) norm (S_R stays well conditioned near convergence)
      launch_axpby_f64(zscale_.as<double>(), Wk, S, nullptr, Wk, S, n_, S, x_.stream);
      DMRG_HIP(hipGetLastError());
    } else if (resp_) {
      // response: the preconditioned right-hand sides (V Psi0)_i / (diag - z_pm)
      double* Sg = Sg_.as<double>();
      launch_axpby_f64(nullptr, rhs_[i], 0, nullptr, Sg, S, n_, S, x_.stream);
      launch_precond_f64(Sg, diag_[i].as<double>(), zsh_.as<double>(), Wk, n_, S, 1e-8, x_.stream);
      DMRG_HIP(hipGetLastError());
    } else {
      tmp.resize(size_t(n_) * S);
      if (guess_ == 1) {
        for (auto& v : tmp) v = rng.normal();
      } else {
        // unit vectors on the n lowest diagonal elements of the middle
        // site's effective Hamiltonian, zero at the other sites
        std::fill(tmp.begin(), tmp.end(), 0.0);
        if (i == L_ / 2) {
          std::vector<double> d(S);
          DMRG_HIP(hipMemcpy(d.data(), diag_[i].p, size_t(S) * 8, hipMemcpyDeviceToHost));
          std::vector<long> idx(S);
          for (long e = 0; e < S; ++e) idx[e] = e;
          const long k = std::min<long>(S, n_ + 1);
          std::partial_sort(idx.begin(), idx.begin() + k, idx.end(), [&](long a, long b) { return d[a] < d[b]; });
          // the lowest element is mostly the reference itself: skip it
          for (int v = 0; v < n_; ++v) tmp[size_t(v) * S + idx[std::min<long>(v + 1, k - 1)]] = 1.0;
        }
      }
      DMRG_HIP(hipMemcpy(Wk, tmp.data(), tmp.size() * 8, hipMemcpyHostToDevice));
    }
    q_c_project(i, Wk, n_);
    copy(Cm + long(m) * S, Wk, long(n_) * S);
    // projected coefficients (eq. cwfn1st)
    double* Ct = Ct_[i].as<double>();
    k_.q_left(i, Cm, Ct, bm_.as<double>(), l);
    // reduced matrices (eqs. hleft2, sleft2)
    double* S0 = S0_.as<double>();
    pc_.mark(PhaseClock::SIG0);
    x_.sigma_general(i, 1, x_.left[i], x_.right[i + 1], Ct, S, S0, S, l, prec_);
    pc_.mark(PhaseClock::VEC);
    gram(Ct, S, l, Ct, S, l, S, SR_.as<double>(), l, 1.0, true);
    gram(Ct, S, l, S0, S, l, S, HR_.as<double>(), l, 1.0, true);
    // response: b_R[mu] = <Psi1^mu | V Psi0> (the left-gauge components of
    // different sites are orthogonal, as for S_R)
    if (resp_) gram(Ct, S, l, rhs_[i], S, 1, S, bR_.as<double>(), 1, 1.0, true);
    gram(Ct, S, l, Dl, S, l, S, HR_.as<double>(), l, 1.0, true);
    gram(Dl, S, l, Ct, S, l, S, HR_.as<double>(), l, 1.0, true);
    if (i == L_ - 1) break;
    // L^(1) (eq. left1st) and the first-order left operators (eq. lopr1st)
    copy(Wk, Ct, long(l) * S);
    k_.scale(i, false, true, Wk, l);
    const int nxt = 1 - cur;
    x_.alloc_opset(FL_[nxt], i + 1, 0, l, true, true, prec_ != DMRG_FP64);
    const double* Li = x_.site[i].L.as<double>();
    pc_.mark(PhaseClock::REN11);
    x_.renorm(DMRG_DIR_LEFT, i, Li, Li, 0, FL_[cur], FL_[nxt], false, l, prec_);
    pc_.mark(PhaseClock::REN01);
    x_.renorm(DMRG_DIR_LEFT, i, Li, Wk, S, x_.left[i], FL_[nxt], true, l, prec_);
    if (rpa_) {
      // <U_v(i+1)| O |L(i+1)> = L^T [<U_v(i)|O|L(i)> x h] L + L^(1)T [<L(i)|O|L(i)> x h] L
      x_.alloc_opset(FLB_[nxt], i + 1, 0, l, true, true, prec_ != DMRG_FP64);
      pc_.mark(PhaseClock::REN11);
      x_.renorm(DMRG_DIR_LEFT, i, Li, Li, 0, FLB_[cur], FLB_[nxt], false, l, prec_);
      pc_.mark(PhaseClock::REN01);
      x_.renorm(DMRG_DIR_LEFT, i, Wk, Li, 0, x_.left[i], FLB_[nxt], true, l, prec_, S);
    }
    pc_.mark(PhaseClock::VEC);
    if (m > 0) copy(Cprev_.as<double>(), Cm, long(m) * S);
    pc_.mark(PhaseClock::HOST);
    x_.sync();
    pc_.mark(PhaseClock::VEC);
    cur = nxt;
  }
  x_.sync();
  FL_[0].data.release();
  FL_[1].data.release();
  FLB_[0].data.release();
  FLB_[1].data.release();
}

void TdaRunner::backward(int l) {
  int cur = 0;
  reserve(FR_, 1, l);
  x_.alloc_opset(FR_[cur], L_, 1, l, true, true, prec_ != DMRG_FP64);
  if (rpa_) {
    reserve(FRB_, 1, l);
    x_.alloc_opset(FRB_[cur], L_, 1, l, true, true, prec_ != DMRG_FP64);
  }
  double* Cb = Cb_.as<double>();
  copy(Cb, Ct_[L_ - 1].as<double>(), long(l) * size(L_ - 1));
  for (int i = L_ - 1; i >= 0; --i) {
    if (p_.verbose >= 2) std::fprintf(stderr, "[tda] backward site %d (l=%d)\n", i, l);
    const long S = size(i);
    const double* Ri = x_.site[i].R.as<double>();
    // R^(1) (eq. right1st): Lambda^-1 C (1 - R^T R)
    double* R1 = R1_[i].as<double>();
    k_.q_right(i, Cb, R1, bm_.as<double>(), l);
    k_.scale(i, true, true, R1, l);
    // first-order right part of the sigma contracted with C^(0)
    pc_.mark(PhaseClock::SIG1);
    x_.sigma_general(i, 1, x_.left[i], FR_[cur], x_.site[i].C.as<double>(), 0, G_[i].as<double>(), S, l, prec_);
    if (rpa_) {
      // Gamma^R_i[v] = <l n V_v| H |Psi0>, and eq. bmatrix: the pairs with
      // the first-order left piece of u at site i and every first-order
      // right piece of v at sites > i, W_half[u][v] += C~_i^u . Gamma^R_i[v]
      // (C~ the Q^L-projected coefficients of eq. cwfn1st of the forward
      // sweep); W = W_half + W_half^T
      x_.sigma_general(i, 1, x_.left[i], FRB_[cur], x_.site[i].C.as<double>(), 0, GB_[i].as<double>(), S, l,
                       prec_);
      gram(Ct_[i].as<double>(), S, l, GB_[i].as<double>(), S, l, S, WR_.as<double>(), l, 1.0, i != L_ - 1);
    }
    pc_.mark(PhaseClock::VEC);
    if (i == 0) break;
    // first-order right operators (eq. ropr1st)
    const int nxt = 1 - cur;
    x_.alloc_opset(FR_[nxt], i, 1, l, true, true, prec_ != DMRG_FP64);
    pc_.mark(PhaseClock::REN11);
    x_.renorm(DMRG_DIR_RIGHT, i, Ri, Ri, 0, FR_[cur], FR_[nxt], false, l, prec_);
    pc_.mark(PhaseClock::REN01);
    x_.renorm(DMRG_DIR_RIGHT, i, Ri, R1, S, x_.right[i + 1], FR_[nxt], true, l, prec_);
    if (rpa_) {
      x_.alloc_opset(FRB_[nxt], i, 1, l, true, true, prec_ != DMRG_FP64);
      pc_.mark(PhaseClock::REN11);
      x_.renorm(DMRG_DIR_RIGHT, i, Ri, Ri, 0, FRB_[cur], FRB_[nxt], false, l, prec_);
      pc_.mark(PhaseClock::REN01);
      x_.renorm(DMRG_DIR_RIGHT, i, R1, Ri, 0, x_.right[i + 1], FRB_[nxt], true, l, prec_, S);
    }
    pc_.mark(PhaseClock::VEC);
    // gauge shift to site i-1 (eq. gauge_bwd): C_{i-1} = C~_{i-1} + L_{i-1} (C_i R_i^T)
    double* Wk = Wk_.as<double>();
    copy(Wk, Ct_[i - 1].as<double>(), long(l) * size(i - 1));
    k_.rmul(i - 1, true, x_.site[i - 1].L.as<double>(), 0, bm_.as<double>(), k_.bm_size[i], Wk, l);
    copy(Cb, Wk, long(l) * size(i - 1));
    pc_.mark(PhaseClock::HOST);
    x_.sync();
    pc_.mark(PhaseClock::VEC);
    cur = nxt;
  }
  x_.sync();
  FR_[0].data.release();
  FR_[1].data.release();
  FRB_[0].data.release();
  FRB_[1].data.release();
}

}  // namespace dmrg

namespace dmrg {

void TdaRunner::run(double* omega, double* etot, double* resid2, int* iters, bool* converged) {
  const auto run0 = std::chrono::steady_clock::now();
  // reference energy E0 = <Psi0|H|Psi0> at site 0
  {
    const double* C0 = x_.site[0].C.as<double>();
    x_.sigma_general(0, 1, x_.left[0], x_.right[1], C0, 0, Wk_.as<double>(), size(0), 1, DMRG_FP64);
    gram(C0, size(0), 1, Wk_.as<double>(), size(0), 1, size(0), tmpd_.as<double>(), 1, 1.0, false);
    DMRG_HIP(hipMemcpy(&E0_, tmpd_.p, 8, hipMemcpyDeviceToHost));
  }
  for (int i = 0; i < L_; ++i) x_.diag(i, 1, diag_[i].as<double>());
  x_.prebuild_tda_plans();
  if (resp_) {
    // shifts of the +omega and -omega components (eqs. realresp, imagresp)
    std::vector<double> z(64, 0.0), nz(64, 0.0);
    z[0] = E0_ - omega_;
    z[1] = E0_ + omega_;
    nz[0] = -z[0];
    nz[1] = -z[1];
    DMRG_HIP(hipMemcpy(zsh_.p, z.data(), 64 * 8, hipMemcpyHostToDevice));
    DMRG_HIP(hipMemcpy(negw_.p, nz.data(), 64 * 8, hipMemcpyHostToDevice));
  }
  std::vector<double> r2;
  // initial trial vectors (unit vectors on the lowest diagonal elements of
  // the middle site, or random components at every site), Q^C projected,
  // then the right-gauge objects and the first reduced matrices
  forward(0, 0, true, uint64_t(p_.seed) * 7919 + 1, r2);
  backward(n_);
  r2.clear();
  int lcur = n_, m = n_;
  bool conv = false;
  int it = 0;
  std::vector<double> w(64), last_w(n_, 0.0);
  // FP32 and BF16x3 runs end with FP64 iterations, switched on near the
  // residual floor of their contractions: a relative error eps on sigma
  // vectors of size ~|E0| at each of the L sites gives sum_i |r_i|^2 ~
  // L (eps E0)^2, with eps = 2^-16 for the split products and 2^-19 for FP32
  // (unit roundoff grown over sums of ~10^3 terms), times 4 for margin; also
  // when the residual meets tol, or stalls for four iterations within a
  // factor 100 of that floor.  The excitation energies are first order in
  // the contraction error of H_R, so only FP64 iterations reach the 1e-5 Eh
  // scale when |E0| is hundreds of Eh.
  const bool can_polish = prec_ != DMRG_FP64 && p_.polish == 0;
  bool polishing = false;
  int polish_iters = 0, stall = 0;
  double best = 1e300;
  const double eps = prec_ == DMRG_BF16X3 ? std::ldexp(1.0, -16) : std::ldexp(1.0, -19);
  const double floor_est = 4.0 * L_ * std::pow(eps * E0_, 2);
  x_.stats.tda_polish_iters = 0;
  x_.stats.tda_hist_len = 0;
  pc_.s = x_.stream;
  pc_.on = p_.verbose >= 1;
  for (int k = 0; k < PhaseClock::N; ++k) x_.stats.tda_phase_ms[k] = 0;
  for (it = 1; it <= p_.max_iter; ++it) {
    auto t0 = std::chrono::steady_clock::now();
    for (double& a : pc_.acc) a = 0;
    pc_.mark(PhaseClock::VEC);
    if (rpa_) {
      // reduced RPA problem (eq. reducedrpa) on the host; sets alpha, the
      // residual coefficients and shifts, and m
      rpa_step(lcur, m);
      for (int v = 0; v < nr_; ++v) w[v] = E0_ + rpa_omega_[v];
    } else {
      // small generalized eigenproblem H_R a = w S_R a (eq. eigs)
      launch_gep_f64(HR_.as<double>(), SR_.as<double>(), lcur, 1e-10, w_.as<double>(), alpha_.as<double>(),
                     rank_.as<int>(), x_.stream);
      DMRG_HIP(hipGetLastError());
      int rank = 0;
      DMRG_HIP(hipMemcpy(w.data(), w_.p, size_t(lcur) * 8, hipMemcpyDeviceToHost));
      DMRG_HIP(hipMemcpy(&rank, rank_.p, sizeof(int), hipMemcpyDeviceToHost));
      // (response mode: the Ritz vectors are a basis, not the roots; the two
      // components coincide at omega = 0 and their corrections are then
      // dependent, which the rank threshold absorbs)
      DMRG_REQUIRE(rank >= (resp_ ? 1 : n_), DMRG_ERR_SINGULAR, "trial space lost rank below the number of roots");
      m = std::min(m, rank);
      if (resp_) {
        response_step(lcur, rank, m, w);
      } else {
        std::vector<double> nw(64, 0.0);
        for (int v = 0; v < n_; ++v) nw[v] = -w[v];
        DMRG_HIP(hipMemcpy(negw_.p, nw.data(), 64 * 8, hipMemcpyHostToDevice));
      }
    }
    for (int v = 0; v < (rpa_ ? nr_ : n_); ++v) last_w[v] = w[v];
    std::vector<double> zs(64, 1.0);
    for (int v = 0; v < n_; ++v) zs[v] = r2.empty() ? 1.0 : 1.0 / std::sqrt(std::max(r2[v], 1e-300));
    DMRG_HIP(hipMemcpy(zscale_.p, zs.data(), 64 * 8, hipMemcpyHostToDevice));
    forward(m, lcur, false, 0, r2);
    const int l = m + n_;
    lcur_last_ = l;
    backward(l);
    pc_.mark(PhaseClock::VEC);
    x_.sync();
    pc_.collect();
    for (int k = 0; k < PhaseClock::N; ++k) x_.stats.tda_phase_ms[k] = pc_.acc[k];
    double mx = 0;
    for (double v : r2) mx = std::max(mx, v);
    auto t1 = std::chrono::steady_clock::now();
    x_.stats.tda_iter_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    x_.stats.tda_iters = it;
    if (it <= DMRG_TDA_HIST) {
      x_.stats.tda_r2_hist[it - 1] = mx;
      x_.stats.tda_hist_len = it;
    }
    if (polishing) x_.stats.tda_polish_iters = ++polish_iters;
    {
      std::string js = resp_ ? "{\"event\": \"response_iteration\""
                             : (rpa_ ? "{\"event\": \"rpa_iteration\"" : "{\"event\": \"tda_iteration\"");
      char buf[512];
      std::snprintf(buf, sizeof buf,
                    ", \"iteration\": %d, \"trial_vectors\": %d, \"max_r2\": %.6g, \"%s\": %.15g, \"%s\": %.15g, "
                    "\"prec\": %d, \"fp64_polish\": %s, \"ms\": %.3f",
                    it, l, mx, resp_ ? "chi_plus" : "omega0", resp_ ? chi_[0] : w[0] - E0_,
                    resp_ ? "chi_minus" : "E0", resp_ ? chi_[1] : E0_, prec_, polishing ? "true" : "false",
                    x_.stats.tda_iter_ms);
      js += buf;
      if (pc_.on) {
        const double* a = pc_.acc;
        std::snprintf(buf, sizeof buf,
                      ", \"phase_ms\": {\"sigma1\": %.3f, \"sigma0\": %.3f, \"ren11\": %.3f, \"ren01\": %.3f, "
                      "\"vec\": %.3f, \"host\": %.3f}",
                      a[0], a[1], a[2], a[3], a[4], a[5]);
        js += buf;
      }
      log_jsonl(js + "}");
    }
    if (p_.verbose) {
      const double* a = pc_.acc;
      std::fprintf(stderr,
                   "[tda] it %d l %d max|r|^2 %.3e  w0 %.10f (%.1f ms: sigma1 %.0f sigma0 %.0f ren11 %.0f ren01 %.0f "
                   "vec %.0f host %.0f)%s\n",
                   it, l, mx, w[0] - E0_, x_.stats.tda_iter_ms, a[0], a[1], a[2], a[3], a[4], a[5],
                   polishing ? " fp64 polish" : "");
    }
    bool done = mx < p_.tol;
    if (can_polish && !polishing) {
      if (mx < 0.5 * best) {
        best = mx;
        stall = 0;
      } else {
        ++stall;
      }
      if (done || mx < floor_est || (stall >= 4 && mx < 100.0 * floor_est)) {
        polishing = true;
        prec_ = DMRG_FP64;
        done = false;
      }
    }
    if (done && (!polishing || polish_iters >= 2)) {
      conv = true;
      break;
    }
    lcur = l;
    // thick restart: when the space is full keep the lowest Ritz vectors,
    // half of the space (at least the n wanted ones and n/2, at least 2, of
    // the next, so that a root close to the edge of the window keeps its
    // neighbour)
    m = (l + n_ <= Nmax_) ? l : std::min(l, std::min(Nmax_ - n_, std::max(n_ + std::max(2, n_ / 2), Nmax_ / 2)));
  }
  // (RPA: per root, the larger of the X and Y residuals)
  for (int v = 0; v < (rpa_ ? nr_ : n_); ++v) {
    etot[v] = last_w[v];
    omega[v] = last_w[v] - E0_;
    resid2[v] = r2.empty() ? 0.0 : (rpa_ ? std::max(r2[v], r2[v + nr_]) : r2[v]);
  }
  *iters = std::min(it, p_.max_iter);
  *converged = conv;
  // reduced matrices of the last forward sweep (test support)
  {
    const int l = lcur_last_;
    x_.tda_l = l;
    x_.tda_hr.resize(size_t(l) * l);
    x_.tda_sr.resize(size_t(l) * l);
    if (l > 0) {
      DMRG_HIP(hipMemcpy(x_.tda_hr.data(), HR_.p, size_t(l) * l * 8, hipMemcpyDeviceToHost));
      DMRG_HIP(hipMemcpy(x_.tda_sr.data(), SR_.p, size_t(l) * l * 8, hipMemcpyDeviceToHost));
    }
  }
  x_.stats.tda_total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - run0).count();
}

// First-order block operators through the C-ABI (Sec. III B eq. lopr1st,
// Sec. III D eq. ropr1st).  The input tensors are first projected on the
// complement of the zeroth-order tensor (Q^L for left, Q^R for right), which
// is the gauge condition of the first-order tensors (Sec. II B); the
// first-order sets have no identity channel because of it.
void Ctx::renorm_first(int i, int dir, int nvec, const double* A1, int prec) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(i >= 0 && i < L, DMRG_ERR_INVALID_ARG, "bad site");
  DMRG_REQUIRE(dir == DMRG_DIR_LEFT || dir == DMRG_DIR_RIGHT, DMRG_ERR_INVALID_ARG, "bad direction");
  DMRG_REQUIRE(nvec >= 1 && A1, DMRG_ERR_INVALID_ARG, "first-order renormalization needs nvec >= 1 tensors");
  const bool left_dir = dir == DMRG_DIR_LEFT;
  FirstOrderChain& F = fo_chain[left_dir ? 0 : 1];
  const int side = left_dir ? 0 : 1;
  const bool f32 = prec != DMRG_FP64;
  const bool start = left_dir ? i == 0 : i == L - 1;
  if (start) {
    // the chain starts at the empty block: bond 0 (left) or bond L (right)
    F.cur = 0;
    F.nvec = nvec;
    F.prec = prec;
    F.bond = left_dir ? 0 : L;
    alloc_opset(F.set[0], F.bond, side, nvec, true, true, f32);
    if (F.set[0].per_vec > 0) {
      if (f32) launch_fill_f32(F.set[0].data.as<float>(), F.set[0].per_vec * nvec, stream);
      else launch_fill_f64(F.set[0].ptr(), F.set[0].per_vec * nvec, 0.0, stream);
    }
  } else {
    const int want = left_dir ? i : i + 1;
    DMRG_REQUIRE(F.bond == want, DMRG_ERR_STATE,
                 "the first-order " + std::string(left_dir ? "left" : "right") + " chain is at bond " +
                     std::to_string(F.bond) + ", not at bond " + std::to_string(want) +
                     " (grow it one site at a time from the chain's start site)");
    DMRG_REQUIRE(F.nvec == nvec, DMRG_ERR_INVALID_ARG, "nvec differs from the chain's");
    DMRG_REQUIRE((F.prec != DMRG_FP64) == f32, DMRG_ERR_INVALID_ARG,
                 "precision class (FP64 or FP32 sets) differs from the chain's");
  }
  GaugeKit& K = gauge_kit();
  const long S = K.size[i];
  ws_fo.ensure(this, (size_t(nvec) * S + size_t(nvec) * K.max_bm) * 8);
  double* X = ws_fo.as<double>();
  double* bm = X + size_t(nvec) * S;
  if (left_dir) K.q_left(i, A1, X, bm, nvec);
  else K.q_right(i, A1, X, bm, nvec);
  const int nxt = 1 - F.cur;
  const int nb = left_dir ? i + 1 : i;
  alloc_opset(F.set[nxt], nb, side, nvec, true, true, f32);
  if (left_dir) {
    const double* Li = site[i].L.as<double>();
    renorm(DMRG_DIR_LEFT, i, Li, Li, 0, F.set[F.cur], F.set[nxt], false, nvec, prec);
    renorm(DMRG_DIR_LEFT, i, Li, X, S, left[i], F.set[nxt], true, nvec, prec);
  } else {
    const double* Ri = site[i].R.as<double>();
    renorm(DMRG_DIR_RIGHT, i, Ri, Ri, 0, F.set[F.cur], F.set[nxt], false, nvec, prec);
    renorm(DMRG_DIR_RIGHT, i, Ri, X, S, right[i + 1], F.set[nxt], true, nvec, prec);
  }
  // only the set at the chain's end is kept between calls (stream-ordered
  // release: the renormalizations above are enqueued before it)
  F.set[F.cur].data.release();
  F.cur = nxt;
  F.bond = nb;
  sync();
}

// TDA sigma at site i (Sec. III D): TDA_FULL is eq. sigv1,
//   sigma^mu = H_0^[i] C^mu(1) + [H_mu^L x h_i x H_0^R] C_i^(0)
//                              + [H_0^L x h_i x H_mu^R] C_i^(0)   (eq. sigv2),
// with the first-order sets of the two chains (a part is zero at the chain's
// start: site 0 for the left part, site L-1 for the right part);
// TDA_DH_LEFT is the first line of eq. sigv2 applied to the given vectors,
//   sigma^mu = [H_mu^L x h_i x H_0^R] C^mu.
void Ctx::sigma_tda(int i, int kind, int nvec, const double* Cin, double* Sout, int prec) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(i >= 0 && i < L, DMRG_ERR_INVALID_ARG, "bad site");
  const FirstOrderChain& FL = fo_chain[0];
  const FirstOrderChain& FR = fo_chain[1];
  const bool use_left = i > 0;
  const bool use_right = kind == DMRG_SIGMA_TDA_FULL && i < L - 1;
  auto check = [&](const FirstOrderChain& F, int bond, const char* side) {
    DMRG_REQUIRE(F.bond == bond, DMRG_ERR_STATE,
                 std::string("the first-order ") + side + " chain must be at bond " + std::to_string(bond) +
                     " (dmrg_renormalize with order 1 up to this site)");
    DMRG_REQUIRE(F.nvec == nvec, DMRG_ERR_INVALID_ARG, std::string("nvec differs from the ") + side + " chain's");
    DMRG_REQUIRE(prec != DMRG_FP64 || F.prec == DMRG_FP64, DMRG_ERR_INVALID_ARG,
                 std::string("an FP64 sigma needs FP64 first-order sets (the ") + side + " chain holds FP32)");
  };
  if (use_left) check(FL, i, "left");
  if (use_right) check(FR, i + 1, "right");
  const long S = long(layout(i, 1).size);
  const double* C0 = site[i].C.as<double>();
  // plans outside the timed region
  if (kind == DMRG_SIGMA_TDA_FULL) sigma_plan(i, 1, left[i], right[i + 1]);
  if (use_left) sigma_plan(i, 1, FL.at(), right[i + 1]);
  if (use_right) sigma_plan(i, 1, left[i], FR.at(), nvec > 1);
  const int parts = (kind == DMRG_SIGMA_TDA_FULL) + use_left + use_right;
  if (parts > 1) ws_tda.ensure(this, size_t(nvec) * S * 8);
  double fl = 0, mfl = 0, mby = 0;
  auto acc = [&]() {
    fl += stats.sigma_flops;
    mfl += stats.sigma_main_flops;
    mby += stats.sigma_main_bytes;
  };
  timed_sigma([&] {
    bool first = true;
    auto target = [&]() { return first ? Sout : ws_tda.as<double>(); };
    auto merge = [&]() {
      if (!first) launch_add_f64(ws_tda.as<double>(), Sout, long(nvec) * S, stream);
      first = false;
    };
    if (kind == DMRG_SIGMA_TDA_FULL) {
      sigma_general(i, 1, left[i], right[i + 1], Cin, S, target(), S, nvec, prec);
      acc();
      merge();
    }
    if (use_left) {
      const bool shared = kind == DMRG_SIGMA_TDA_FULL;  // C^(0) for every vector
      sigma_general(i, 1, FL.at(), right[i + 1], shared ? C0 : Cin, shared ? 0 : S, target(), S, nvec, prec);
      acc();
      merge();
    }
    if (use_right) {
      sigma_general(i, 1, left[i], FR.at(), C0, 0, target(), S, nvec, prec);
      acc();
      merge();
    }
    if (first) launch_fill_f64(Sout, long(nvec) * S, 0.0, stream);  // no part (left part at site 0)
    DMRG_HIP(hipGetLastError());
  });
  stats.sigma_flops = fl;
  stats.sigma_main_flops = mfl;
  stats.sigma_main_bytes = mby;
}

void Ctx::tda_roots(int nroots, const dmrg_davidson_params& p, double* omega, double* etot, double* resid2,
                    int* iters, bool* converged) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(omega && etot && resid2 && iters && converged, DMRG_ERR_INVALID_ARG, "null outputs");
  DMRG_REQUIRE(p.max_iter >= 1, DMRG_ERR_INVALID_ARG, "max_iter must be >= 1");
  // the run builds its own first-order operators; the chains of
  // dmrg_renormalize (order 1) are released first to bound the peak memory
  sync();
  for (auto& f : fo_chain) f.reset();
  {
    TdaRunner r(*this, nroots, p);
    r.run(omega, etot, resid2, iters, converged);
  }
  release_workspaces();
}

// DMRG-RPA roots (Sec. II C eq. dmrgrpa, Sec. III E): the TDA sweeps with
// the second-order matrix W accumulated in the backward sweep (eq.
// bmatrix) and the reduced non-Hermitian problem of eq. reducedrpa.
void Ctx::rpa_roots(int nroots, const dmrg_davidson_params& p, double* omega, double* etot, double* resid2,
                    int* iters, bool* converged) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(omega && etot && resid2 && iters && converged, DMRG_ERR_INVALID_ARG, "null outputs");
  DMRG_REQUIRE(p.max_iter >= 1, DMRG_ERR_INVALID_ARG, "max_iter must be >= 1");
  DMRG_REQUIRE(nroots >= 1, DMRG_ERR_INVALID_ARG, "need nroots >= 1");
  sync();
  for (auto& f : fo_chain) f.reset();
  {
    TdaRunner r(*this, nroots, p, nullptr, true);
    r.run(omega, etot, resid2, iters, converged);
  }
  release_workspaces();
}

void Ctx::export_host(MpsHostCopy& m) {
  size_t sz[4] = {0, 0, 0, 0};
  export_mps(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, sz);
  m.nsec.assign(L + 1, 0);
  m.sec.assign(3 * sz[0], 0);
  m.L.assign(sz[1], 0.0);
  m.R.assign(sz[1], 0.0);
  m.C.assign(sz[1], 0.0);
  m.lam.assign(sz[3], 0.0);
  export_mps(m.nsec.data(), m.sec.data(), m.L.data(), m.R.data(), m.C.data(), m.lam.data(), sz);
}

// V Psi0 projected on every site, P_i^T V Psi0 (flat one-site layouts at the
// offsets off[i]), for the one-body operator V = sum_pq v_pq E_pq (v need not
// be symmetric): the zeroth-order sigma of a second context that holds V
// (no two-body part) on the same MPS, applied to C_i^(0).
void Ctx::onebody_rhs(const double* v, const MpsHostCopy& m, double* rhs, const std::vector<long>& off) {
  const std::vector<double> zero(size_t(L) * L * L * L, 0.0);
  Ctx vc(L, Na, Nb, v, zero.data(), 0.0, device, stream, &allocator);
  vc.import_mps(m.nsec.data(), m.sec.data(), m.L.data(), m.R.data(), m.C.data(), m.lam.data());
  vc.build_ops(DMRG_FP64);
  for (int i = 0; i < L; ++i) vc.sigma(i, 1, 1, site[i].C.as<double>(), rhs + off[i], DMRG_FP64);
  vc.sync();
}

// DMRG-TDA roots and their one-particle transition densities
// gamma^nu_pq = <Psi^nu | E_pq | Psi0> (E_pq the spin-summed excitation
// operator; Sec. VI A): the TDA run of dmrg_tda_roots, then for every (p, q)
// the site projections of E_pq Psi0 contracted with the roots' left-gauge
// components.  gamma[(nu L + p) L + q].
void Ctx::tda_transition(int nroots, const dmrg_davidson_params& p, double* omega, double* etot, double* resid2,
                         int* iters, bool* converged, double* gamma) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(omega && etot && resid2 && iters && converged && gamma, DMRG_ERR_INVALID_ARG, "null outputs");
  DMRG_REQUIRE(p.max_iter >= 1, DMRG_ERR_INVALID_ARG, "max_iter must be >= 1");
  sync();
  for (auto& f : fo_chain) f.reset();
  std::vector<long> off(L + 1, 0);
  for (int i = 0; i < L; ++i) off[i + 1] = off[i] + layout(i, 1).size;
  MpsHostCopy mc;
  export_host(mc);
  DBuf rhs;
  rhs.alloc(this, size_t(std::max<long>(off[L], 1)) * 8);
  std::vector<const double*> ptr;
  for (int i = 0; i < L; ++i) ptr.push_back(rhs.as<double>() + off[i]);
  {
    TdaRunner r(*this, nroots, p);
    r.run(omega, etot, resid2, iters, converged);
    std::vector<double> e(size_t(L) * L, 0.0), ov(nroots);
    for (int a = 0; a < L; ++a)
      for (int b = 0; b < L; ++b) {
        std::fill(e.begin(), e.end(), 0.0);
        e[size_t(a) * L + b] = 1.0;
        onebody_rhs(e.data(), mc, rhs.as<double>(), off);
        r.root_overlaps(ptr, ov.data());
        for (int nu = 0; nu < nroots; ++nu) gamma[(size_t(nu) * L + a) * L + b] = ov[nu];
      }
  }
  sync();
  release_workspaces();
}

// Frequency-dependent linear response to a one-body perturbation
// V = sum_pq v_pq E_pq (Sec. II B, eqs. realresp and imagresp; first-order
// wavefunction of eq. psi1st in the gauge of eqs. left-orthoSeb and
// right-orthoSeb).  The right-hand side V Psi0, projected on every site, is
// the zeroth-order sigma of a second context that holds V (no two-body part)
// on the same MPS.  chi[0] = <V Psi0 | Psi1_+omega>, chi[1] = <V Psi0 |
// Psi1_-omega>, with (H - (E0 -+ omega)) Psi1_pm = -Q V Psi0 in the tangent
// space.
void Ctx::response(const double* v, double omega, const dmrg_davidson_params& p, double* chi, double* resid2,
                   int* iters, bool* converged) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(v && chi && resid2 && iters && converged, DMRG_ERR_INVALID_ARG, "null arguments");
  DMRG_REQUIRE(p.max_iter >= 1, DMRG_ERR_INVALID_ARG, "max_iter must be >= 1");
  DMRG_REQUIRE(std::isfinite(omega), DMRG_ERR_INVALID_ARG, "omega must be finite");
  double vmax = 0;
  for (int a = 0; a < L * L; ++a) {
    DMRG_REQUIRE(std::isfinite(v[a]), DMRG_ERR_INVALID_ARG, "non-finite entry in v");
    vmax = std::max(vmax, std::abs(v[a]));
  }
  for (int a = 0; a < L; ++a)
    for (int b = a + 1; b < L; ++b)
      DMRG_REQUIRE(std::abs(v[a * L + b] - v[b * L + a]) <= 1e-12 * std::max(vmax, 1.0), DMRG_ERR_INVALID_ARG,
                   "v must be symmetric");
  sync();
  for (auto& f : fo_chain) f.reset();
  std::vector<long> off(L + 1, 0);
  for (int i = 0; i < L; ++i) off[i + 1] = off[i] + layout(i, 1).size;
  DBuf rhs;
  rhs.alloc(this, size_t(std::max<long>(off[L], 1)) * 8);
  MpsHostCopy mc;
  export_host(mc);
  onebody_rhs(v, mc, rhs.as<double>(), off);
  ResponseSpec rs;
  rs.omega = omega;
  for (int i = 0; i < L; ++i) rs.rhs.push_back(rhs.as<double>() + off[i]);
  {
    TdaRunner r(*this, 2, p, &rs);
    double om[2], et[2];
    r.run(om, et, resid2, iters, converged);
    chi[0] = r.chi(0);
    chi[1] = r.chi(1);
  }
  sync();
  release_workspaces();
}

}  // namespace dmrg
