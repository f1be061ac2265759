// Ground-state DMRG by two-site sweeps (Sec. II A: the site problem of
// eq. dmrg solved on the two-site product basis, then split back into one-site
// tensors; eq. gauge-shift for the moving orthogonality centre).
//
// All tensors stay on the device.  One step at sites (i, i+1):
//   1. two-site guess from the current centre tensor and its neighbour;
//   2. Davidson for the lowest eigenpair of the two-site effective
//      Hamiltonian (sigma = the two-site contraction of the engine, in the
//      requested precision; subspace, projections and residuals in FP64);
//   3. decimation at bond i+1: per symmetry sector q of the bond the block
//      matrix Psi_q (rows (a, n1), columns (n2, c)) is factorized by an SVD on
//      the device, the largest singular values over all sectors are kept
//      (at most M, relative cutoff 1e-12), and the new bond, its Schmidt
//      values and the two one-site tensors are written from U, S, V^T;
//   4. the block operators of the grown block are renormalized.
// After the sweeps one non-truncating one-site pass (SVD of each centre
// tensor, moving right) leaves the mixed-canonical MPS with L_i, C_i, R_i and
// diagonal Lambda at every bond that the DMRG-TDA needs, and the zeroth-order
// operators are rebuilt from it.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <random>

#include "engine.hpp"
#include "kernels.hpp"

namespace dmrg {

namespace {

// host -> device copy of a small list; waits for the stream first because
// the buffer may still be read by earlier work
template <class T>
void put(Ctx& x, DBuf& buf, const std::vector<T>& v) {
  x.sync();
  buf.ensure(&x, std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty()) DMRG_HIP(hipMemcpy(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Placement of the row-major blocks of a tensor into per-sector dense
// matrices (column-major) for the SVD.
struct SplitSpec {
  std::vector<QN> q;            // label of each sector
  std::vector<int> rows, cols;  // per sector
  struct Place {
    long off;
    int rows, cols, sec, r0, c0;
  };
  std::vector<Place> places;
};

struct SplitOut {
  std::vector<int> kmax;
  std::vector<long> a_off, u_off, s_off, vt_off;
  std::vector<std::vector<double>> s;  // host singular values per sector
  DBuf A, U, S, VT, E, info;
};

class Ground {
 public:
  Ground(Ctx& x, const dmrg_sweep_params& p) : x_(x), p_(p) {
    DMRG_REQUIRE(rocblas_create_handle(&h_) == rocblas_status_success, DMRG_ERR_INTERNAL, "rocblas handle");
    rocblas_set_stream(h_, x_.stream);
  }
  ~Ground() { rocblas_destroy_handle(h_); }
  void run(double* energy, double* discarded, bool* converged);

 private:
  Ctx& x_;
  dmrg_sweep_params p_;
  rocblas_handle h_;
  DBuf jobs_, psi_, V_, HV_, diag_, tmp_, part_, small_, w_, alpha_, rank_, newL_, newR_, newC_;

  void svd(const double* T, const SplitSpec& sp, SplitOut& o);
  static std::vector<int> truncate(const SplitOut& o, int M, double* discarded);
  void copies(const std::vector<Copy2D>& c);
  void gemm(GemmPlan& P, const std::vector<GJob>& jobs, std::vector<std::vector<GContrib>>& per, const Bases& b);
  double davidson(int i, double* psi, long n, int* iters, int width = 2);
  void random_start(int M0);
  void build_right_ops();
  void step(int i, bool right, int M, double* energy, double* dw);
  void final_pass();
  // non-truncating split of the centre C_i at its right bond (the body of
  // final_pass): L_i, Lambda_{i+1}, C_{i+1} = S V^T R_{i+1}
  void move_right(int i);
  // non-truncating split of the tensor in site[i].R at its left bond:
  // site[i].R becomes R_i, bond i gets the Schmidt values, and the tensor in
  // site[i-1].R is multiplied by U S
  void split_left(int i);
  // one-site sweep (right, then left) optimizing the centre at every site
  double onesite_sweep();
  double gram1(const double* a, const double* b, long n);
};

void Ground::copies(const std::vector<Copy2D>& c) {
  if (c.empty()) return;
  put(x_, jobs_, c);
  launch_copy2d_f64(jobs_.as<Copy2D>(), int(c.size()), x_.stream);
  DMRG_HIP(hipGetLastError());
  x_.sync();  // the job list is reused by the next call
}

void Ground::gemm(GemmPlan& P, const std::vector<GJob>& jobs0, std::vector<std::vector<GContrib>>& per,
                  const Bases& b) {
  std::vector<GJob> jobs = jobs0;
  build_gemm_plan(x_, P, jobs, per);
  P.launch(x_, b, 1);
  x_.sync();
}

double Ground::gram1(const double* a, const double* b, long n) {
  part_.ensure(&x_, std::max<size_t>(size_t(64) * 64 * 64, size_t(gram_parts(n))) * 8);
  small_.ensure(&x_, 64 * 64 * 8);
  launch_gram_f64(a, n, 1, b, n, 1, n, small_.as<double>(), 1, part_.as<double>(), 1.0, false, x_.stream);
  x_.sync();
  double r = 0;
  DMRG_HIP(hipMemcpy(&r, small_.p, 8, hipMemcpyDeviceToHost));
  return r;
}

// Per-sector SVD of the placed blocks: U (rows x kmax), S, V^T (kmax x cols),
// column-major, kmax = min(rows, cols).
void Ground::svd(const double* T, const SplitSpec& sp, SplitOut& o) {
  const int ns = int(sp.q.size());
  o.kmax.assign(ns, 0);
  o.a_off.assign(ns, 0);
  o.u_off.assign(ns, 0);
  o.s_off.assign(ns, 0);
  o.vt_off.assign(ns, 0);
  long na = 0, nu = 0, nsv = 0, nvt = 0;
  int emax = 1;
  for (int s = 0; s < ns; ++s) {
    const int m = sp.rows[s], n = sp.cols[s], k = std::min(m, n);
    o.kmax[s] = k;
    o.a_off[s] = na;
    o.u_off[s] = nu;
    o.s_off[s] = nsv;
    o.vt_off[s] = nvt;
    na += long(m) * n;
    nu += long(m) * k;
    nsv += k;
    nvt += long(k) * n;
    emax = std::max(emax, k);
  }
  o.A.ensure(&x_, std::max<long>(na, 1) * 8);
  o.U.ensure(&x_, std::max<long>(nu, 1) * 8);
  o.S.ensure(&x_, std::max<long>(nsv, 1) * 8);
  o.VT.ensure(&x_, std::max<long>(nvt, 1) * 8);
  o.E.ensure(&x_, size_t(emax) * 8);
  o.info.ensure(&x_, std::max<size_t>(ns, 1) * sizeof(rocblas_int));
  launch_fill_f64(o.A.as<double>(), na, 0.0, x_.stream);
  std::vector<Copy2D> cp;
  for (auto& pl : sp.places) {
    const long ld = sp.rows[pl.sec];
    cp.push_back({T + pl.off, o.A.as<double>() + o.a_off[pl.sec] + pl.r0 + long(pl.c0) * ld, long(pl.cols), 1, 1,
                  ld, nullptr, pl.rows, pl.cols, 0, 0});
  }
  copies(cp);
  for (int s = 0; s < ns; ++s) {
    const int m = sp.rows[s], n = sp.cols[s], k = o.kmax[s];
    if (k == 0) continue;
    rocblas_status st = rocsolver_dgesvd(h_, rocblas_svect_singular, rocblas_svect_singular, m, n,
                                         o.A.as<double>() + o.a_off[s], m, o.S.as<double>() + o.s_off[s],
                                         o.U.as<double>() + o.u_off[s], m, o.VT.as<double>() + o.vt_off[s], k,
                                         o.E.as<double>(), rocblas_outofplace, o.info.as<rocblas_int>() + s);
    DMRG_REQUIRE(st == rocblas_status_success, DMRG_ERR_INTERNAL, "rocsolver_dgesvd failed");
  }
  std::vector<double> sv(std::max<long>(nsv, 1));
  std::vector<rocblas_int> info(std::max(ns, 1));
  x_.sync();
  DMRG_HIP(hipMemcpy(sv.data(), o.S.p, size_t(nsv) * 8, hipMemcpyDeviceToHost));
  DMRG_HIP(hipMemcpy(info.data(), o.info.p, size_t(ns) * sizeof(rocblas_int), hipMemcpyDeviceToHost));
  o.s.assign(ns, {});
  for (int s = 0; s < ns; ++s) {
    // empty sectors run no SVD and leave their info entry unwritten
    DMRG_REQUIRE(o.kmax[s] == 0 || info[s] == 0, DMRG_ERR_NOT_CONVERGED, "SVD of a sector did not converge");
    o.s[s].assign(sv.begin() + o.s_off[s], sv.begin() + o.s_off[s] + o.kmax[s]);
  }
}

// Keep the largest singular values over all sectors: at most M, none below
// 1e-12 of the largest.  Returns the kept count per sector.
std::vector<int> Ground::truncate(const SplitOut& o, int M, double* discarded) {
  std::vector<std::pair<double, int>> all;
  double tot = 0, mx = 0;
  for (size_t s = 0; s < o.s.size(); ++s)
    for (double v : o.s[s]) {
      all.push_back({v, int(s)});
      tot += v * v;
      mx = std::max(mx, v);
    }
  std::stable_sort(all.begin(), all.end(), [](auto& a, auto& b) { return a.first > b.first; });
  std::vector<int> k(o.s.size(), 0);
  double kept = 0;
  for (size_t t = 0; t < all.size() && int(t) < M; ++t) {
    if (all[t].first <= 1e-12 * mx) break;
    k[all[t].second]++;
    kept += all[t].first * all[t].first;
  }
  if (discarded) *discarded = tot > 0 ? std::max(0.0, 1.0 - kept / tot) : 0.0;
  return k;
}

// Lowest eigenpair of the two-site effective Hamiltonian at (i, i+1); psi
// (n elements) is the start vector on entry and the normalized Ritz vector
// on exit.
double Ground::davidson(int i, double* psi, long n, int* iters, int width) {
  const int nmax = int(std::min<long>(16, n));
  V_.ensure(&x_, size_t(nmax) * n * 8);
  HV_.ensure(&x_, size_t(nmax) * n * 8);
  diag_.ensure(&x_, size_t(n) * 8);
  tmp_.ensure(&x_, size_t(2) * n * 8);
  part_.ensure(&x_, std::max<size_t>(size_t(64) * 64 * 64, size_t(gram_parts(n)) * nmax * nmax) * 8);
  small_.ensure(&x_, 64 * 64 * 8 * 2);
  w_.ensure(&x_, 64 * 8);
  alpha_.ensure(&x_, 64 * 64 * 8);
  rank_.ensure(&x_, 16);
  double* V = V_.as<double>();
  double* HV = HV_.as<double>();
  double* Hs = small_.as<double>();
  double* Ss = Hs + 64 * 64;
  x_.diag(i, width, diag_.as<double>());
  // v0 = psi / |psi|
  const double nrm = std::sqrt(gram1(psi, psi, n));
  DMRG_REQUIRE(nrm > 0, DMRG_ERR_INTERNAL, "zero start vector");
  std::vector<double> one{1.0 / nrm};
  DBuf& sc = newC_;
  put(x_, sc, one);
  launch_axpby_f64(sc.as<double>(), psi, 0, nullptr, V, 0, 1, n, x_.stream);
  int k = 1, it = 0;
  double theta = 0;
  auto add_sigma = [&](int j) {
    x_.sigma_general(i, width, x_.left[i], x_.right[i + width], V + long(j) * n, n, HV + long(j) * n, n, 1,
                     p_.prec);
  };
  add_sigma(0);
  for (;;) {
    ++it;
    // projected matrices over the (orthonormal) basis
    launch_gram_f64(V, n, k, HV, n, k, n, Hs, k, part_.as<double>(), 1.0, false, x_.stream);
    launch_gram_f64(V, n, k, V, n, k, n, Ss, k, part_.as<double>(), 1.0, false, x_.stream);
    launch_gep_f64(Hs, Ss, k, 1e-12, w_.as<double>(), alpha_.as<double>(), rank_.as<int>(), x_.stream);
    DMRG_HIP(hipGetLastError());
    x_.sync();
    DMRG_HIP(hipMemcpy(&theta, w_.p, 8, hipMemcpyDeviceToHost));
    // Ritz vector x = V a, Hx = HV a, residual r = Hx - theta x
    double* xv = tmp_.as<double>();
    double* hx = xv + n;
    launch_rotate_f64(V, n, k, alpha_.as<double>(), k, 1, xv, n, n, x_.stream);
    launch_rotate_f64(HV, n, k, alpha_.as<double>(), k, 1, hx, n, n, x_.stream);
    std::vector<double> coef{-theta, 1.0};
    put(x_, sc, coef);
    // hx <- hx - theta x (the residual)
    launch_axpby_f64(sc.as<double>(), xv, 0, sc.as<double>() + 1, hx, 0, 1, n, x_.stream);
    const double r2 = gram1(hx, hx, n);
    if (p_.verbose >= 3) std::fprintf(stderr, "[ground]   site %d it %d E %.12f |r|^2 %.2e\n", i, it, theta, r2);
    if (r2 < p_.davidson_tol || it >= std::max(1, p_.davidson_max_iter) || k >= n) {
      const double xn = std::sqrt(gram1(xv, xv, n));
      std::vector<double> s1{1.0 / xn};
      put(x_, sc, s1);
      launch_axpby_f64(sc.as<double>(), xv, 0, nullptr, psi, 0, 1, n, x_.stream);
      DMRG_HIP(hipGetLastError());
      *iters = it;
      return theta;
    }
    // correction t = r / (diag - theta), orthogonalized against V
    double* t = V + long(std::min(k, nmax - 1)) * n;
    if (k == nmax) {
      // restart from the Ritz vector
      DMRG_HIP(hipMemcpyAsync(V, xv, size_t(n) * 8, hipMemcpyDeviceToDevice, x_.stream));
      add_sigma(0);
      k = 1;
      t = V + n;
    } else {
      t = V + long(k) * n;
    }
    std::vector<double> th{theta};
    put(x_, sc, th);
    launch_precond_f64(hx, diag_.as<double>(), sc.as<double>(), t, 1, n, 1e-8, x_.stream);
    for (int pass = 0; pass < 2; ++pass) {
      launch_gram_f64(V, n, k, t, n, 1, n, Ss, 1, part_.as<double>(), 1.0, false, x_.stream);
      launch_rotate_f64(V, n, k, Ss, k, 1, hx, n, n, x_.stream);
      std::vector<double> c2{-1.0, 1.0};
      put(x_, sc, c2);
      launch_axpby_f64(sc.as<double>(), hx, 0, sc.as<double>() + 1, t, 0, 1, n, x_.stream);
    }
    const double tn = std::sqrt(gram1(t, t, n));
    if (tn < 1e-14) {
      *iters = it;
      const double xn = std::sqrt(gram1(xv, xv, n));
      std::vector<double> s1{1.0 / xn};
      put(x_, sc, s1);
      launch_axpby_f64(sc.as<double>(), xv, 0, nullptr, psi, 0, 1, n, x_.stream);
      return theta;
    }
    std::vector<double> s2{1.0 / tn};
    put(x_, sc, s2);
    launch_axpby_f64(sc.as<double>(), t, 0, nullptr, t, 0, 1, n, x_.stream);
    add_sigma(k);
    ++k;
  }
}

// Sector of bond `bond` reached from sector a of bond `bond-1` with local
// state n, or -1.
int next_sector(const Bond& bl, int a, const Bond& br, int n) {
  const QN d = site_qn(n);
  return br.find(QN{bl.q[a].na + d.na, bl.q[a].nb + d.nb});
}

// New bond from the kept counts: sectors with k > 0, in label order (the
// split sectors are already sorted), Schmidt values normalized.
void kept_bond(const SplitSpec& sp, const SplitOut& o, const std::vector<int>& k, Bond& nb,
               std::vector<std::vector<double>>& lam, std::vector<int>& newidx, std::vector<double>& sflat,
               std::vector<long>& soff) {
  double nrm = 0;
  for (size_t s = 0; s < k.size(); ++s)
    for (int j = 0; j < k[s]; ++j) nrm += o.s[s][j] * o.s[s][j];
  nrm = std::sqrt(nrm);
  nb = Bond();
  lam.clear();
  newidx.assign(k.size(), -1);
  sflat.clear();
  soff.assign(k.size(), 0);
  for (size_t s = 0; s < k.size(); ++s) {
    if (k[s] == 0) continue;
    newidx[s] = int(nb.q.size());
    nb.idx[sp.q[s].key()] = int(nb.q.size());
    nb.q.push_back(sp.q[s]);
    nb.dim.push_back(k[s]);
    std::vector<double> l(o.s[s].begin(), o.s[s].begin() + k[s]);
    for (double& v : l) v /= nrm;
    soff[s] = long(sflat.size());
    sflat.insert(sflat.end(), l.begin(), l.end());
    lam.push_back(std::move(l));
  }
}

void Ground::build_right_ops() {
  const int L = x_.L;
  const int rp = p_.prec == DMRG_BF16X3 ? DMRG_FP32 : p_.prec;
  x_.left.resize(L + 1);
  x_.right.resize(L + 1);
  x_.alloc_opset(x_.left[0], 0, 0, 1, false);
  x_.alloc_opset(x_.right[L], L, 1, 1, false);
  for (int i = L - 1; i >= 1; --i) {
    x_.alloc_opset(x_.right[i], i, 1, 1, false);
    x_.renorm(DMRG_DIR_RIGHT, i, x_.site[i].R.as<double>(), x_.site[i].R.as<double>(), 0, x_.right[i + 1],
              x_.right[i], false, 1, rp);
  }
  x_.ops_prec = p_.prec;
}

// Random start: sectors of every bond with dimensions min(exact, M0 / #sectors),
// Gaussian tensors, made right-canonical by SVDs from the right; the
// centre C_0 is normalized.
void Ground::random_start(int M0) {
  const int L = x_.L, Na = x_.Na, Nb = x_.Nb;
  auto binom = [](int n, int k) -> double {
    if (k < 0 || k > n) return 0;
    double r = 1;
    for (int j = 1; j <= k; ++j) r = r * (n - k + j) / j;
    return r;
  };
  std::vector<Bond> B(L + 1);
  for (int b = 0; b <= L; ++b) {
    std::vector<std::pair<QN, double>> secs;
    for (int na = std::max(0, Na - (L - b)); na <= std::min(b, Na); ++na)
      for (int nb = std::max(0, Nb - (L - b)); nb <= std::min(b, Nb); ++nb) {
        const double ex = std::min(binom(b, na) * binom(b, nb), binom(L - b, Na - na) * binom(L - b, Nb - nb));
        if (ex >= 1) secs.push_back({QN{na, nb}, ex});
      }
    const int per = std::max(1, M0 / std::max<int>(1, int(secs.size())));
    for (auto& q : secs) {
      B[b].idx[q.first.key()] = int(B[b].q.size());
      B[b].q.push_back(q.first);
      B[b].dim.push_back(int(std::min<double>(q.second, per)));
    }
  }
  x_.have_mps = true;
  x_.bonds = B;
  x_.lam.assign(L + 1, {});
  for (int b = 0; b <= L; ++b)
    for (int d : x_.bonds[b].dim) x_.lam[b].push_back(std::vector<double>(d, 1.0));
  x_.lam_dev.clear();
  x_.laminv_dev.clear();
  for (int b = 0; b <= L; ++b) x_.invalidate_bond(b);
  x_.left.clear();
  x_.right.clear();
  x_.site.clear();
  x_.site.resize(L);
  std::mt19937_64 rng(uint64_t(p_.seed) * 2654435761ull + 17);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int i = 0; i < L; ++i) {
    const SiteLayout& S = x_.layout(i, 1);
    std::vector<double> v(S.size);
    for (double& e : v) e = nd(rng);
    put(x_, x_.site[i].R, v);
  }
  // right-canonicalize: split site i at its left bond
  for (int i = L - 1; i >= 1; --i) split_left(i);
  // centre C_0 = T_0 / |T_0|
  const SiteLayout& S0 = x_.layout(0, 1);
  const double nrm = std::sqrt(gram1(x_.site[0].R.as<double>(), x_.site[0].R.as<double>(), long(S0.size)));
  std::vector<double> sc{1.0 / nrm};
  DBuf d;
  put(x_, d, sc);
  x_.site[0].C.alloc(&x_, std::max<size_t>(S0.size, 1) * 8);
  launch_axpby_f64(d.as<double>(), x_.site[0].R.as<double>(), 0, nullptr, x_.site[0].C.as<double>(), 0, 1,
                   long(S0.size), x_.stream);
  x_.sync();
  x_.lam[0] = {{1.0}};
  x_.lam_dev.clear();
  x_.laminv_dev.clear();
  x_.lam_dev.resize(L + 1);
  x_.laminv_dev.resize(L + 1);
  for (int b = 0; b <= L; ++b) x_.upload_lambda_bond(b);
}

void Ground::split_left(int i) {
  const SiteLayout Si = x_.layout(i, 1);
  const SiteLayout Sp = x_.layout(i - 1, 1);
  const Bond bl = x_.bonds[i];
  SplitSpec sp;
  sp.q = bl.q;
  sp.rows = bl.dim;
  sp.cols.assign(bl.q.size(), 0);
  std::map<std::pair<int, int>, int> c0;  // (n, c) within sector a
  for (auto& b : Si.blk) {
    auto key = std::make_pair(b.a * 64 + b.n, b.c);
    c0[key] = sp.cols[b.a];
    sp.places.push_back({long(b.off), b.rows, b.cols, b.a, 0, sp.cols[b.a]});
    sp.cols[b.a] += b.cols;
  }
  SplitOut o;
  svd(x_.site[i].R.as<double>(), sp, o);
  std::vector<int> k = truncate(o, 1 << 30, nullptr);
  Bond nb;
  std::vector<std::vector<double>> lam;
  std::vector<int> ni;
  std::vector<double> sflat;
  std::vector<long> soff;
  kept_bond(sp, o, k, nb, lam, ni, sflat, soff);
  // raw (unnormalized) singular values scale the carried part
  std::vector<double> sraw;
  std::vector<long> sroff(k.size(), 0);
  for (size_t q = 0; q < k.size(); ++q) {
    sroff[q] = long(sraw.size());
    sraw.insert(sraw.end(), o.s[q].begin(), o.s[q].begin() + k[q]);
  }
  DBuf sdev;
  put(x_, sdev, sraw);
  // US = U scaled by S (column-major, ld = rows)
  DBuf us;
  us.ensure(&x_, std::max<size_t>(o.U.bytes / 8, 1) * 8);
  std::vector<Copy2D> cp;
  for (size_t q = 0; q < k.size(); ++q)
    if (k[q] > 0)
      cp.push_back({o.U.as<double>() + o.u_off[q], us.as<double>() + o.u_off[q], 1, long(sp.rows[q]), 1,
                    long(sp.rows[q]), sdev.as<double>() + sroff[q], sp.rows[q], k[q], 2, 0});
  copies(cp);
  DBuf oldp = std::move(x_.site[i - 1].R);
  x_.set_bond(i, nb, lam);
  const SiteLayout& Ni = x_.layout(i, 1);
  const SiteLayout& Np = x_.layout(i - 1, 1);
  // R_i = rows of V^T
  x_.site[i].R.alloc(&x_, std::max<size_t>(Ni.size, 1) * 8);
  launch_fill_f64(x_.site[i].R.as<double>(), long(Ni.size), 0.0, x_.stream);
  cp.clear();
  for (auto& b : Ni.blk) {
    const int q = bl.find(nb.q[b.a]);
    // locate the old column block (n, c): same n, c index unchanged (bond i+1)
    auto it = c0.find(std::make_pair(q * 64 + b.n, b.c));
    if (it == c0.end()) continue;
    cp.push_back({o.VT.as<double>() + o.vt_off[q] + long(it->second) * o.kmax[q],
                  x_.site[i].R.as<double>() + b.off, 1, long(o.kmax[q]), long(b.cols), 1, nullptr, b.rows, b.cols,
                  0, 0});
  }
  copies(cp);
  // carry: T_{i-1}(a', n', a) <- T_{i-1}(a', n', a_old) (U S)_a
  x_.site[i - 1].R.alloc(&x_, std::max<size_t>(Np.size, 1) * 8);
  std::vector<GJob> jobs;
  std::vector<std::vector<GContrib>> per;
  for (auto& b : Np.blk) {
    GJob j{};
    j.offC = long(b.off);
    j.baseC = B_SOUT;
    j.ldc = b.cols;
    j.m = b.rows;
    j.n = b.cols;
    jobs.push_back(j);
    per.emplace_back();
    const int q = bl.find(nb.q[b.c]);  // old sector of bond i
    const int ob = Sp.find(b.a, b.n);
    if (q < 0 || ob < 0 || Sp.blk[ob].c != q) continue;
    per.back().push_back({long(Sp.blk[ob].off), o.u_off[q], Sp.blk[ob].cols, sp.rows[q], sp.rows[q], GC_TRANS_B,
                          B_AKET, B_AUX, 1.0});
  }
  Bases bs{};
  bs.p[B_AKET] = oldp.as<double>();
  bs.p[B_AUX] = us.as<double>();
  bs.p[B_SOUT] = x_.site[i - 1].R.as<double>();
  GemmPlan P;
  gemm(P, jobs, per, bs);
}

// One two-site step at (i, i+1); right: the centre moves to i+1.
void Ground::step(int i, bool right, int M, double* energy, double* dw) {
  const int rp = p_.prec == DMRG_BF16X3 ? DMRG_FP32 : p_.prec;
  const SiteLayout S2 = x_.layout(i, 2);  // bonds i and i+2: unchanged by the step
  const long n = long(S2.size);
  psi_.ensure(&x_, std::max<long>(n, 1) * 8);
  {
    const SiteLayout& A = x_.layout(i, 1);
    const SiteLayout& Bl = x_.layout(i + 1, 1);
    std::vector<GJob> jobs;
    std::vector<std::vector<GContrib>> per;
    for (auto& b : S2.blk) {
      GJob j{};
      j.offC = long(b.off);
      j.baseC = B_SOUT;
      j.ldc = b.cols;
      j.m = b.rows;
      j.n = b.cols;
      jobs.push_back(j);
      per.emplace_back();
      const int ab = A.find(b.a, b.n / 4);
      if (ab < 0) continue;
      const int bb = Bl.find(A.blk[ab].c, b.n % 4);
      if (bb < 0 || Bl.blk[bb].c != b.c) continue;
      per.back().push_back({long(A.blk[ab].off), long(Bl.blk[bb].off), A.blk[ab].cols, Bl.blk[bb].cols,
                            A.blk[ab].cols, 0, B_AKET, B_AUX, 1.0});
    }
    Bases bs{};
    bs.p[B_AKET] = right ? x_.site[i].C.as<double>() : x_.site[i].L.as<double>();
    bs.p[B_AUX] = right ? x_.site[i + 1].R.as<double>() : x_.site[i + 1].C.as<double>();
    bs.p[B_SOUT] = psi_.as<double>();
    GemmPlan P;
    gemm(P, jobs, per, bs);
  }
  int its = 0;
  *energy = davidson(i, psi_.as<double>(), n, &its);
  // split at bond i+1: rows (a, n1), columns (n2, c) per sector
  const Bond& bi = x_.bonds[i];
  std::map<QN, int> secs;
  for (auto& b : S2.blk) {
    const QN d = site_qn(b.n / 4);
    secs[QN{bi.q[b.a].na + d.na, bi.q[b.a].nb + d.nb}] = 0;
  }
  SplitSpec sp;
  for (auto& kv : secs) {
    kv.second = int(sp.q.size());
    sp.q.push_back(kv.first);
  }
  sp.rows.assign(sp.q.size(), 0);
  sp.cols.assign(sp.q.size(), 0);
  std::map<std::tuple<int, int, int>, int> r0, c0;  // (sec, a, n1) / (sec, n2, c)
  for (auto& b : S2.blk) {
    const QN d = site_qn(b.n / 4);
    const int sec = secs[QN{bi.q[b.a].na + d.na, bi.q[b.a].nb + d.nb}];
    auto rk = std::make_tuple(sec, b.a, b.n / 4);
    auto ck = std::make_tuple(sec, b.n % 4, b.c);
    if (!r0.count(rk)) {
      r0[rk] = sp.rows[sec];
      sp.rows[sec] += b.rows;
    }
    if (!c0.count(ck)) {
      c0[ck] = sp.cols[sec];
      sp.cols[sec] += b.cols;
    }
    sp.places.push_back({long(b.off), b.rows, b.cols, sec, r0[rk], c0[ck]});
  }
  SplitOut o;
  svd(psi_.as<double>(), sp, o);
  std::vector<int> k = truncate(o, M, dw);
  Bond nb;
  std::vector<std::vector<double>> lam;
  std::vector<int> ni;
  std::vector<double> sflat;
  std::vector<long> soff;
  kept_bond(sp, o, k, nb, lam, ni, sflat, soff);
  DBuf sdev;
  put(x_, sdev, sflat);
  x_.set_bond(i + 1, nb, lam);
  const SiteLayout& Li = x_.layout(i, 1);
  const SiteLayout& Ri = x_.layout(i + 1, 1);
  const Bond& bn = x_.bonds[i + 1];
  DBuf& dl = right ? x_.site[i].L : x_.site[i].C;       // left factor (U or U S)
  DBuf& dr = right ? x_.site[i + 1].C : x_.site[i + 1].R;  // right factor (S V^T or V^T)
  dl.alloc(&x_, std::max<size_t>(Li.size, 1) * 8);
  dr.alloc(&x_, std::max<size_t>(Ri.size, 1) * 8);
  launch_fill_f64(dl.as<double>(), long(Li.size), 0.0, x_.stream);
  launch_fill_f64(dr.as<double>(), long(Ri.size), 0.0, x_.stream);
  std::vector<Copy2D> cp;
  for (auto& b : Li.blk) {
    const int sec = secs[bn.q[b.c]];
    auto it = r0.find(std::make_tuple(sec, b.a, b.n));
    if (it == r0.end()) continue;
    cp.push_back({o.U.as<double>() + o.u_off[sec] + it->second, dl.as<double>() + b.off, 1, long(sp.rows[sec]),
                  long(b.cols), 1, right ? nullptr : sdev.as<double>() + soff[sec], b.rows, b.cols, right ? 0 : 2, 0});
  }
  for (auto& b : Ri.blk) {
    const int sec = secs[bn.q[b.a]];
    auto it = c0.find(std::make_tuple(sec, b.n, b.c));
    if (it == c0.end()) continue;
    cp.push_back({o.VT.as<double>() + o.vt_off[sec] + long(it->second) * o.kmax[sec], dr.as<double>() + b.off, 1,
                  long(o.kmax[sec]), long(b.cols), 1, right ? sdev.as<double>() + soff[sec] : nullptr, b.rows,
                  b.cols, right ? 1 : 0, 0});
  }
  copies(cp);
  if (right) {
    x_.alloc_opset(x_.left[i + 1], i + 1, 0, 1, false);
    x_.renorm(DMRG_DIR_LEFT, i, x_.site[i].L.as<double>(), x_.site[i].L.as<double>(), 0, x_.left[i], x_.left[i + 1],
              false, 1, rp);
  } else {
    x_.alloc_opset(x_.right[i + 1], i + 1, 1, 1, false);
    x_.renorm(DMRG_DIR_RIGHT, i + 1, x_.site[i + 1].R.as<double>(), x_.site[i + 1].R.as<double>(), 0,
              x_.right[i + 2], x_.right[i + 1], false, 1, rp);
  }
  x_.sync();
  if (p_.verbose >= 2)
    std::fprintf(stderr, "[ground] %s site %d E %.12f davidson %d its, bond %d dim %d, discarded %.2e\n",
                 right ? "->" : "<-", i, *energy, its, i + 1, bn.total(), *dw);
}

void Ground::move_right(int i) {
  const SiteLayout Si = x_.layout(i, 1);
  const SiteLayout Sn = x_.layout(i + 1, 1);
  const Bond bo = x_.bonds[i + 1];
  SplitSpec sp;
  sp.q = bo.q;
  sp.rows.assign(bo.q.size(), 0);
  sp.cols = bo.dim;
  std::map<std::pair<int, int>, int> r0;  // (a, n) -> row offset in sector c
  for (auto& b : Si.blk) {
    r0[{b.a, b.n}] = sp.rows[b.c];
    sp.places.push_back({long(b.off), b.rows, b.cols, b.c, sp.rows[b.c], 0});
    sp.rows[b.c] += b.rows;
  }
  SplitOut o;
  svd(x_.site[i].C.as<double>(), sp, o);
  std::vector<int> k = truncate(o, 1 << 30, nullptr);
  Bond nb;
  std::vector<std::vector<double>> lam;
  std::vector<int> ni;
  std::vector<double> sflat;
  std::vector<long> soff;
  kept_bond(sp, o, k, nb, lam, ni, sflat, soff);
  DBuf sdev;
  put(x_, sdev, sflat);
  DBuf oldR_i = std::move(x_.site[i].R), oldR_n = std::move(x_.site[i + 1].R);
  if (i == 0) oldR_i = DBuf();
  x_.set_bond(i + 1, nb, lam);
  const SiteLayout& Ni = x_.layout(i, 1);
  const SiteLayout& Nn = x_.layout(i + 1, 1);
  const Bond& bn = x_.bonds[i + 1];
  for (auto* d : {&x_.site[i].L, &x_.site[i].C}) {
    d->alloc(&x_, std::max<size_t>(Ni.size, 1) * 8);
    launch_fill_f64(d->as<double>(), long(Ni.size), 0.0, x_.stream);
  }
  std::vector<Copy2D> cp;
  for (auto& b : Ni.blk) {
    const int sec = bo.find(bn.q[b.c]);
    auto it = r0.find({b.a, b.n});
    if (sec < 0 || it == r0.end()) continue;
    for (int w = 0; w < 2; ++w)
      cp.push_back({o.U.as<double>() + o.u_off[sec] + it->second,
                    (w ? x_.site[i].C : x_.site[i].L).as<double>() + b.off, 1, long(sp.rows[sec]), long(b.cols), 1,
                    w ? sdev.as<double>() + soff[sec] : nullptr, b.rows, b.cols, w ? 2 : 0, 0});
  }
  copies(cp);
  // R_i <- R_i V (i >= 1); R_0 = C_0
  x_.site[i].R.alloc(&x_, std::max<size_t>(Ni.size, 1) * 8);
  if (i == 0) {
    DMRG_HIP(hipMemcpyAsync(x_.site[0].R.p, x_.site[0].C.p, Ni.size * 8, hipMemcpyDeviceToDevice, x_.stream));
  } else {
    std::vector<GJob> jobs;
    std::vector<std::vector<GContrib>> per;
    for (auto& b : Ni.blk) {
      GJob j{};
      j.offC = long(b.off);
      j.baseC = B_SOUT;
      j.ldc = b.cols;
      j.m = b.rows;
      j.n = b.cols;
      jobs.push_back(j);
      per.emplace_back();
      const int sec = bo.find(bn.q[b.c]);
      const int ob = Si.find(b.a, b.n);
      if (sec < 0 || ob < 0) continue;
      // V(c_old, c_new) = VT[c_new + c_old * kmax]: row-major K x N with ldb = kmax
      per.back().push_back({long(Si.blk[ob].off), o.vt_off[sec], Si.blk[ob].cols, o.kmax[sec], Si.blk[ob].cols, 0,
                            B_AKET, B_AUX, 1.0});
    }
    Bases bs{};
    bs.p[B_AKET] = oldR_i.as<double>();
    bs.p[B_AUX] = o.VT.as<double>();
    bs.p[B_SOUT] = x_.site[i].R.as<double>();
    GemmPlan P;
    gemm(P, jobs, per, bs);
  }
  // R_{i+1} <- V^T R_{i+1}, C_{i+1} = S R_{i+1}
  x_.site[i + 1].R.alloc(&x_, std::max<size_t>(Nn.size, 1) * 8);
  x_.site[i + 1].C.alloc(&x_, std::max<size_t>(Nn.size, 1) * 8);
  {
    std::vector<GJob> jobs;
    std::vector<std::vector<GContrib>> per;
    for (auto& b : Nn.blk) {
      GJob j{};
      j.offC = long(b.off);
      j.baseC = B_SOUT;
      j.ldc = b.cols;
      j.m = b.rows;
      j.n = b.cols;
      jobs.push_back(j);
      per.emplace_back();
      const int sec = bo.find(bn.q[b.a]);
      const int ob = Sn.find(sec, b.n);
      if (sec < 0 || ob < 0 || Sn.blk[ob].c != b.c) continue;
      // op(A) = V^T (k x m_old): A^T with A row-major m_old x kmax
      per.back().push_back({o.vt_off[sec], long(Sn.blk[ob].off), o.kmax[sec], Sn.blk[ob].cols, Sn.blk[ob].rows,
                            GC_TRANS_A, B_AUX, B_AKET, 1.0});
    }
    Bases bs{};
    bs.p[B_AKET] = oldR_n.as<double>();
    bs.p[B_AUX] = o.VT.as<double>();
    bs.p[B_SOUT] = x_.site[i + 1].R.as<double>();
    GemmPlan P;
    gemm(P, jobs, per, bs);
  }
  cp.clear();
  for (auto& b : Nn.blk) {
    const int sec = bo.find(bn.q[b.a]);
    cp.push_back({x_.site[i + 1].R.as<double>() + b.off, x_.site[i + 1].C.as<double>() + b.off, long(b.cols), 1,
                  long(b.cols), 1, sdev.as<double>() + soff[sec], b.rows, b.cols, 1, 0});
  }
  copies(cp);
}

// Non-truncating one-site pass from the centre at site 0 to the right:
// C_i = U S V^T at bond i+1 gives L_i = U, Lambda_{i+1} = S, C_i = U S,
// R_i <- R_i V and R_{i+1} <- V^T R_{i+1}, C_{i+1} = S R_{i+1}.
void Ground::final_pass() {
  const int L = x_.L;
  for (int i = 0; i + 1 < L; ++i) move_right(i);
  // last site: bond L has one state, L_{L-1} = C_{L-1}
  const SiteLayout& Sl = x_.layout(L - 1, 1);
  x_.site[L - 1].L.alloc(&x_, std::max<size_t>(Sl.size, 1) * 8);
  DMRG_HIP(hipMemcpyAsync(x_.site[L - 1].L.p, x_.site[L - 1].C.p, Sl.size * 8, hipMemcpyDeviceToDevice, x_.stream));
  x_.lam[0] = {{1.0}};
  x_.lam[L] = {{1.0}};
  x_.upload_lambda();
  x_.sync();
}

// One-site sweep (eq. dmrg on the one-site product basis, Sec. II A),
// right then left, from the centre at site 0: at every site the lowest
// eigenvector of H_0^[i] replaces the centre, which then moves on by a
// non-truncating split.  The bond dimensions stay fixed, so repeated sweeps
// converge to a stationary point of the energy on the MPS manifold of the
// current bonds, which the two-site sweeps (they truncate after every step)
// do not reach.  Ends with the centre at site 0, R_1..R_{L-1} and the right
// operators of every bond consistent.  Returns the last local eigenvalue.
double Ground::onesite_sweep() {
  const int L = x_.L;
  const int rp = p_.prec == DMRG_BF16X3 ? DMRG_FP32 : p_.prec;
  double e = 0;
  int its = 0;
  auto copy = [&](DBuf& dst, const DBuf& src, long n) {
    dst.alloc(&x_, std::max<size_t>(size_t(n), 1) * 8);
    if (n > 0) DMRG_HIP(hipMemcpyAsync(dst.p, src.p, size_t(n) * 8, hipMemcpyDeviceToDevice, x_.stream));
  };
  for (int i = 0; i < L; ++i) {
    e = davidson(i, x_.site[i].C.as<double>(), long(x_.layout(i, 1).size), &its, 1);
    if (i + 1 == L) break;
    move_right(i);
    x_.alloc_opset(x_.left[i + 1], i + 1, 0, 1, false);
    x_.renorm(DMRG_DIR_LEFT, i, x_.site[i].L.as<double>(), x_.site[i].L.as<double>(), 0, x_.left[i], x_.left[i + 1],
              false, 1, rp);
    x_.sync();
  }
  for (int i = L - 1; i >= 1; --i) {
    // split the optimized centre at its left bond and carry U S into L_{i-1}
    copy(x_.site[i].R, x_.site[i].C, long(x_.layout(i, 1).size));
    copy(x_.site[i - 1].R, x_.site[i - 1].L, long(x_.layout(i - 1, 1).size));
    split_left(i);
    const long np = long(x_.layout(i - 1, 1).size);
    copy(x_.site[i - 1].C, x_.site[i - 1].R, np);
    x_.alloc_opset(x_.right[i], i, 1, 1, false);
    x_.renorm(DMRG_DIR_RIGHT, i, x_.site[i].R.as<double>(), x_.site[i].R.as<double>(), 0, x_.right[i + 1],
              x_.right[i], false, 1, rp);
    x_.sync();
    e = davidson(i - 1, x_.site[i - 1].C.as<double>(), np, &its, 1);
  }
  return e;
}

void Ground::run(double* energy, double* discarded, bool* converged) {
  const int L = x_.L;
  DMRG_REQUIRE(p_.nsweeps >= 1 && p_.M_schedule, DMRG_ERR_INVALID_ARG, "need nsweeps >= 1 and a bond schedule");
  for (int s = 0; s < p_.nsweeps; ++s) DMRG_REQUIRE(p_.M_schedule[s] >= 1, DMRG_ERR_INVALID_ARG, "bad M");
  DMRG_REQUIRE(L >= 2, DMRG_ERR_INVALID_ARG, "need at least two sites");
  DMRG_REQUIRE(p_.onesite_sweeps >= 0, DMRG_ERR_INVALID_ARG, "onesite_sweeps must be >= 0");
  if (!x_.have_mps) random_start(p_.M_schedule[0]);
  build_right_ops();
  double e = 0, last = 0, dwmax = 0;
  for (int sw = 0; sw < p_.nsweeps; ++sw) {
    const auto t0 = std::chrono::steady_clock::now();
    const int M = p_.M_schedule[sw];
    dwmax = 0;
    for (int i = 0; i + 1 < L; ++i) {
      double dw = 0;
      step(i, true, M, &e, &dw);
      dwmax = std::max(dwmax, dw);
    }
    for (int i = L - 2; i >= 0; --i) {
      double dw = 0;
      step(i, false, M, &e, &dw);
      dwmax = std::max(dwmax, dw);
    }
    if (p_.verbose >= 1)
      std::fprintf(stderr, "[ground] sweep %d M %d E %.12f dE %.2e max discarded %.2e\n", sw, M, e, e - last, dwmax);
    {
      char buf[320];
      std::snprintf(buf, sizeof buf,
                    "{\"event\": \"ground_sweep\", \"sweep\": %d, \"M\": %d, \"energy\": %.15g, \"dE\": %.6g, "
                    "\"max_discarded\": %.6g, \"prec\": %d, \"seconds\": %.4f}",
                    sw, M, e, sw ? e - last : 0.0, dwmax, p_.prec,
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
      log_jsonl(buf);
    }
    last = e;
  }
  for (int k = 0; k < p_.onesite_sweeps; ++k) {
    const auto t0 = std::chrono::steady_clock::now();
    e = onesite_sweep();
    if (p_.verbose >= 1) std::fprintf(stderr, "[ground] one-site sweep %d E %.14f dE %.2e\n", k, e, e - last);
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "{\"event\": \"onesite_sweep\", \"sweep\": %d, \"energy\": %.15g, \"dE\": %.6g, \"seconds\": %.4f}",
                  k, e, e - last, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    log_jsonl(buf);
    last = e;
  }
  final_pass();
  // the operator pools of the returned state are built in FP64, so that the
  // reported <Psi|H|Psi> (and the DMRG-TDA reference built on it) carries no
  // contraction rounding of the sweeps' precision
  x_.build_ops(DMRG_FP64);
  // <Psi|H|Psi> in FP64 at site 0
  const SiteLayout& S0 = x_.layout(0, 1);
  DBuf sig;
  sig.alloc(&x_, std::max<size_t>(S0.size, 1) * 8);
  x_.sigma(0, 1, 1, x_.site[0].C.as<double>(), sig.as<double>(), DMRG_FP64);
  const double nn = gram1(x_.site[0].C.as<double>(), x_.site[0].C.as<double>(), long(S0.size));
  *energy = gram1(x_.site[0].C.as<double>(), sig.as<double>(), long(S0.size)) / nn;
  if (discarded) *discarded = dwmax;
  *converged = true;
}

}  // namespace

void Ctx::sweep_ground(const dmrg_sweep_params& p, double* energy, double* discarded, bool* converged) {
  require_gpu();
  {
    Ground g(*this, p);
    g.run(energy, discarded, converged);
  }
  release_workspaces();
}

}  // namespace dmrg
