// Channel classification of the ab initio Hamiltonian and generation of the
// site tensors W_b (see qc_mpo.hpp for the channel table).
#include "qc_mpo.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>
#include <tuple>

namespace dmrg {

namespace {
inline int site_of(int m) { return m >> 1; }
inline int spin_of(int m) { return m & 1; }

// sign of the stable sort of a sequence by group label (count inversions)
inline int sort_sign(const int* g, int n) {
  int inv = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (g[i] > g[j]) ++inv;
  return (inv & 1) ? -1 : 1;
}
}  // namespace

QCHamiltonian::QCHamiltonian(int L, const double* h, const double* eri, double ecore, double screen)
    : L_(L), switch_(L / 2), ecore_(ecore) {
  if (L < 2 || L > 128) throw std::invalid_argument("number of sites out of range");
  build_terms(h, eri, screen);
  build_strings(1);
  build_strings(2);
  build_channels();
}

void QCHamiltonian::build_terms(const double* h, const double* eri, double screen) {
  const int L = L_, nm = 2 * L;
  auto E = [&](int p, int q, int r, int s) { return eri[((size_t(p) * L + q) * L + r) * L + s]; };
  terms_.clear();
  // one-body: a+_{p s} a_{q s}
  for (int p = 0; p < L; ++p)
    for (int q = 0; q < L; ++q) {
      double t = h[p * L + q];
      if (std::fabs(t) <= screen) continue;
      for (int s = 0; s < 2; ++s) {
        Term T{};
        T.c = t;
        T.n = 2;
        T.op[0] = {1, int16_t(2 * p + s)};
        T.op[1] = {0, int16_t(2 * q + s)};
        terms_.push_back(T);
      }
    }
  // two-body: 1/2 sum g_PQRS a+_P a+_Q a_R a_S with g_PQRS = (iP iS|iQ iR) d(sP,sS) d(sQ,sR);
  // collected on P<Q, R<S with W_PQRS = g_PQRS - g_QPRS.
  auto g = [&](int P, int Q, int R, int S) -> double {
    if (spin_of(P) != spin_of(S) || spin_of(Q) != spin_of(R)) return 0.0;
    return E(site_of(P), site_of(S), site_of(Q), site_of(R));
  };
  for (int P = 0; P < nm; ++P)
    for (int Q = P + 1; Q < nm; ++Q)
      for (int R = 0; R < nm; ++R)
        for (int S = R + 1; S < nm; ++S) {
          if (spin_of(P) + spin_of(Q) != spin_of(R) + spin_of(S)) continue;
          double w = g(P, Q, R, S) - g(Q, P, R, S);
          if (std::fabs(w) <= screen) continue;
          Term T{};
          T.c = w;
          T.n = 4;
          T.op[0] = {1, int16_t(P)};
          T.op[1] = {1, int16_t(Q)};
          T.op[2] = {0, int16_t(R)};
          T.op[3] = {0, int16_t(S)};
          terms_.push_back(T);
        }
  terms_on_site_.assign(L, {});
  for (size_t t = 0; t < terms_.size(); ++t) {
    Term& T = terms_[t];
    T.smin = L;
    T.smax = -1;
    for (int k = 0; k < T.n; ++k) {
      T.smin = std::min(T.smin, site_of(T.op[k].m));
      T.smax = std::max(T.smax, site_of(T.op[k].m));
    }
    int last = -1;
    std::vector<int> s;
    for (int k = 0; k < T.n; ++k) s.push_back(site_of(T.op[k].m));
    std::sort(s.begin(), s.end());
    for (int x : s)
      if (x != last) {
        terms_on_site_[x].push_back(int(t));
        last = x;
      }
  }
}

void QCHamiltonian::build_strings(int width) {
  const int nm = 2 * width, d = 1 << nm;  // d = 4^width
  auto occ = [&](int n, int j) -> int {
    int site = j >> 1, spin = j & 1;
    int ns = (width == 1) ? n : (site == 0 ? n / 4 : n % 4);
    return (ns >> spin) & 1;
  };
  auto bits_of = [&](int n) {
    int b = 0;
    for (int j = 0; j < nm; ++j) b |= occ(n, j) << j;
    return b;
  };
  std::vector<int> state_of_bits(d);
  for (int n = 0; n < d; ++n) state_of_bits[bits_of(n)] = n;
  auto& S = strings_[width - 1];
  auto& idx = string_index_[width - 1];
  S.clear();
  for (int cm = 0; cm < (1 << nm); ++cm)
    for (int dm = 0; dm < (1 << nm); ++dm) {
      DotString ds;
      ds.cre_mask = cm;
      ds.des_mask = dm;
      ds.parity = (__builtin_popcount(cm) + __builtin_popcount(dm)) & 1;
      ds.dna = ds.dnb = 0;
      for (int j = 0; j < nm; ++j) {
        int sgn = ((cm >> j) & 1) - ((dm >> j) & 1);
        if (j & 1) ds.dnb += sgn; else ds.dna += sgn;
      }
      for (int ket = 0; ket < d; ++ket) {
        int b = bits_of(ket);
        double sign = 1.0;
        bool ok = true;
        for (int j = nm - 1; j >= 0 && ok; --j)  // annihilators, rightmost (largest) first
          if ((dm >> j) & 1) {
            if (!((b >> j) & 1)) { ok = false; break; }
            if (__builtin_popcount(b & ((1 << j) - 1)) & 1) sign = -sign;
            b ^= 1 << j;
          }
        for (int j = nm - 1; j >= 0 && ok; --j)  // creators, rightmost (largest) first
          if ((cm >> j) & 1) {
            if ((b >> j) & 1) { ok = false; break; }
            if (__builtin_popcount(b & ((1 << j) - 1)) & 1) sign = -sign;
            b ^= 1 << j;
          }
        if (!ok) continue;
        ds.ket.push_back(ket);
        ds.bra.push_back(state_of_bits[b]);
        ds.val.push_back(sign);
      }
      idx[cm * (1 << nm) + dm] = int(S.size());
      S.push_back(ds);
    }
}

int QCHamiltonian::string_id(int width, int cm, int dm) const {
  return string_index_[width - 1].at(cm * (1 << (2 * width)) + dm);
}

uint64_t QCHamiltonian::classify(const Lad* ops, int n, int b, int mode, int* nleft) const {
  Lad X[4], Y[4];
  int nx = 0, ny = 0;
  for (int k = 0; k < n; ++k) {
    if (site_of(ops[k].m) < b) X[nx++] = ops[k];
    else Y[ny++] = ops[k];
  }
  if (nleft) *nleft = nx;
  if (ny == 0) return chan_key(CH_H_ID, -1, -1);
  if (nx == 0) return chan_key(CH_ID_H, -1, -1);
  if (nx == 1) return chan_key(X[0].cre ? CH_CRE_L : CH_DES_L, X[0].m, -1);
  if (ny == 1) return chan_key(Y[0].cre ? CH_T_CRE : CH_T_DES, Y[0].m, -1);
  // two and two
  if (mode == 0) {
    if (X[0].cre && X[1].cre) return chan_key(CH_AA, X[0].m, X[1].m);
    if (!X[0].cre && !X[1].cre) return chan_key(CH_DD, X[0].m, X[1].m);
    return chan_key(CH_AD, X[0].m, X[1].m);
  }
  if (!Y[0].cre && !Y[1].cre) return chan_key(CH_PP, Y[0].m, Y[1].m);
  if (Y[0].cre && Y[1].cre) return chan_key(CH_PPB, Y[0].m, Y[1].m);
  return chan_key(CH_QQ, Y[0].m, Y[1].m);
}

Channel QCHamiltonian::describe(uint64_t key, int) const {
  Channel c{};
  c.key = key;
  int t = key_type(key), p = key_p(key), q = key_q(key);
  auto add = [&](int m, int s) {
    if (spin_of(m)) c.dnb += s; else c.dna += s;
  };
  switch (t) {
    case CH_ID_H: c.parity = 0; c.compl_left = false; break;
    case CH_H_ID: c.parity = 0; c.compl_left = true; break;
    case CH_CRE_L: add(p, +1); c.parity = 1; c.compl_left = false; break;
    case CH_DES_L: add(p, -1); c.parity = 1; c.compl_left = false; break;
    case CH_T_CRE: add(p, -1); c.parity = 1; c.compl_left = true; break;
    case CH_T_DES: add(p, +1); c.parity = 1; c.compl_left = true; break;
    case CH_AA: add(p, +1); add(q, +1); c.parity = 0; c.compl_left = false; break;
    case CH_DD: add(p, -1); add(q, -1); c.parity = 0; c.compl_left = false; break;
    case CH_AD: add(p, +1); add(q, -1); c.parity = 0; c.compl_left = false; break;
    case CH_PP: add(p, +1); add(q, +1); c.parity = 0; c.compl_left = true; break;
    case CH_PPB: add(p, -1); add(q, -1); c.parity = 0; c.compl_left = true; break;
    case CH_QQ: add(p, -1); add(q, +1); c.parity = 0; c.compl_left = true; break;
    default: throw std::logic_error("bad channel type");
  }
  return c;
}

void QCHamiltonian::build_channels() {
  const int L = L_;
  for (int mode = 0; mode < 2; ++mode) {
    // mode 0 serves bonds 0..switch+1, mode 1 bonds switch+1..L
    const int b0 = mode == 0 ? 0 : std::min(switch_ + 1, L);
    const int b1 = mode == 0 ? std::min(switch_ + 1, L) : L;
    std::vector<std::vector<uint64_t>> keys(L + 1);
    for (int b = b0; b <= b1; ++b) {
      if (b < L) keys[b].push_back(chan_key(CH_ID_H, -1, -1));
      if (b > 0) keys[b].push_back(chan_key(CH_H_ID, -1, -1));
    }
    for (const Term& T : terms_)
      for (int b = std::max(T.smin + 1, b0); b <= std::min(T.smax, b1); ++b)
        keys[b].push_back(classify(T.op, T.n, b, mode, nullptr));
    bonds_[mode].assign(L + 1, {});
    for (int b = 0; b <= L; ++b) {
      BondChannels& B = bonds_[mode][b];
      B.mode = (b >= b0 && b <= b1) ? mode : -1;
      if (B.mode < 0) continue;
      auto& k = keys[b];
      std::sort(k.begin(), k.end());
      k.erase(std::unique(k.begin(), k.end()), k.end());
      for (uint64_t key : k) {
        B.idx[key] = int(B.ch.size());
        B.ch.push_back(describe(key, b));
      }
    }
  }
}

const BondChannels& QCHamiltonian::channels(int b, int mode) const {
  if (b < 0 || b > L_ || mode < 0 || mode > 1 || bonds_[mode][b].mode != mode)
    throw std::invalid_argument("no channel set for this bond and pair mode");
  return bonds_[mode][b];
}

const SiteOp& QCHamiltonian::site_op(int b, int width, int m0, int m1) {
  const int64_t ck = int64_t(b) * 16 + width * 4 + m0 * 2 + m1;
  {
    // built outside the lock; a concurrent builder of the same key keeps the
    // first entry (element references stay valid across rehashing)
    std::lock_guard<std::mutex> lock(cache_mu_);
    auto it = cache_.find(ck);
    if (it != cache_.end()) return it->second;
  }
  if (width < 1 || width > 2 || b < 0 || b + width > L_ || m0 > m1) throw std::invalid_argument("bad dot");
  const BondChannels& B0 = channels(b, m0);
  const BondChannels& B1 = channels(b + width, m1);
  const int lo = 2 * b, hi = 2 * (b + width);  // dot modes [lo, hi)
  struct Acc { double c; bool set; };
  std::map<std::tuple<int, int, int>, Acc> acc;
  auto put = [&](int src, int dst, int sid, double v, bool set) {
    auto key = std::make_tuple(src, dst, sid);
    auto f = acc.find(key);
    if (f == acc.end()) {
      acc[key] = {v, set};
      return;
    }
    if (set || f->second.set) {
      if (!(set && f->second.set) || std::fabs(f->second.c - v) > 1e-12)
        throw std::logic_error("inconsistent channel factorization");
      return;
    }
    f->second.c += v;
  };
  // 1. pass-through channels (same key on both sides, no operator on the dot)
  for (size_t w = 0; w < B0.ch.size(); ++w) {
    int w2 = B1.find(B0.ch[w].key);
    if (w2 >= 0) put(int(w), w2, 0, 1.0, true);
  }
  auto handle = [&](const Term& T) {
    int grp[4], g1[4], g2[4];
    Lad Xp[4], Yp[4];
    int nxp = 0, nyp = 0, cm = 0, dm = 0;
    for (int k = 0; k < T.n; ++k) {
      int m = T.op[k].m;
      grp[k] = m < lo ? 0 : (m < hi ? 1 : 2);
      if (grp[k] == 1) {
        if (T.op[k].cre) cm |= 1 << (m - lo); else dm |= 1 << (m - lo);
      }
    }
    const int s3 = sort_sign(grp, T.n);
    // signs of the partial reorderings
    int ny = 0, nx = 0;
    for (int k = 0; k < T.n; ++k) {
      if (grp[k] >= 1) g1[ny++] = grp[k];      // Y part at bond b: D then R'
      if (grp[k] <= 1) g2[nx++] = grp[k];      // X' part at bond b+width: L then D
    }
    const int s_r = sort_sign(g1, ny);
    const int s_l = sort_sign(g2, nx);
    (void)Xp; (void)Yp; (void)nxp; (void)nyp;
    uint64_t k0 = classify(T.op, T.n, b, B0.mode, nullptr);
    uint64_t k1 = classify(T.op, T.n, b + width, B1.mode, nullptr);
    int w0 = B0.find(k0), w1 = B1.find(k1);
    if (w0 < 0 || w1 < 0) throw std::logic_error("term classified into a missing channel");
    int sid = string_id(width, cm, dm);
    if (B0.ch[w0].compl_left) put(w0, w1, sid, double(s_r), true);
    else if (!B1.ch[w1].compl_left) put(w0, w1, sid, double(s_l), true);
    else put(w0, w1, sid, T.c * s3, false);
  };
  // 2. terms with an operator on the dot
  std::vector<int> seen;
  for (int s = b; s < b + width; ++s)
    for (int t : terms_on_site_[s]) seen.push_back(t);
  std::sort(seen.begin(), seen.end());
  seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
  for (int t : seen) handle(terms_[t]);
  // 3. switch from normal-left to normal-right pairs across the dot
  if (B0.mode == 0 && B1.mode == 1) {
    for (const Term& T : terms_) {
      if (T.n != 4) continue;
      int nl = 0, nd = 0;
      for (int k = 0; k < 4; ++k) {
        int m = T.op[k].m;
        if (m < lo) ++nl; else if (m < hi) ++nd;
      }
      if (nl == 2 && nd == 0) handle(T);
    }
  }
  // 4. the constant enters once, on the first site
  if (b == 0 && ecore_ != 0.0) {
    int w0 = B0.find(chan_key(CH_ID_H, -1, -1)), w1 = B1.find(chan_key(CH_H_ID, -1, -1));
    put(w0, w1, 0, ecore_, false);
  }
  SiteOp op;
  op.b = b;
  op.width = width;
  op.d = 1 << (2 * width);
  for (auto& kv : acc) {
    if (kv.second.c == 0.0) continue;
    op.e.push_back({std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second.c});
  }
  std::lock_guard<std::mutex> lock(cache_mu_);
  return cache_.emplace(ck, std::move(op)).first->second;
}

}  // namespace dmrg
