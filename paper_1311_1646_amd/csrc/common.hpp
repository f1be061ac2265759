// Shared host-side definitions: error handling, device buffers, symmetry
// sectors and block layouts.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dmrg.h"

namespace dmrg {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define DMRG_HIP(call)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::dmrg::Error(DMRG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define DMRG_REQUIRE(cond, code, msg) \
  do {                                \
    if (!(cond)) throw ::dmrg::Error(code, msg); \
  } while (0)

// particle-number label of a sector
struct QN {
  int na, nb;
  bool operator<(const QN& o) const { return na != o.na ? na < o.na : nb < o.nb; }
  bool operator==(const QN& o) const { return na == o.na && nb == o.nb; }
  int key() const { return (na + 256) * 1024 + (nb + 256); }
  int n() const { return na + nb; }
};

// local basis of one site: 0:|0>, 1:|a>, 2:|b>, 3:|ab>
inline QN site_qn(int n) { return QN{n & 1, n >> 1}; }
inline QN dot_qn(int n, int width) {
  if (width == 1) return site_qn(n);
  QN a = site_qn(n / 4), b = site_qn(n % 4);
  return QN{a.na + b.na, a.nb + b.nb};
}

struct Bond {
  std::vector<QN> q;
  std::vector<int> dim;
  std::unordered_map<int, int> idx;
  int find(QN x) const {
    auto it = idx.find(x.key());
    return it == idx.end() ? -1 : it->second;
  }
  int total() const {
    int t = 0;
    for (int d : dim) t += d;
    return t;
  }
};

// Coefficient tensor of a dot of width 1 or 2 starting at site i:
// blocks (a at bond i, n in [0,d), c at bond i+width), row-major m_a x m_c.
struct SiteLayout {
  int site = 0, width = 1, d = 4;
  struct Blk { int a, n, c, rows, cols; size_t off; };
  std::vector<Blk> blk;
  std::vector<int> lookup;  // a*d + n -> block id or -1
  size_t size = 0;
  int find(int a, int n) const { return lookup[size_t(a) * d + n]; }
};

// Block-sparse operator on the states of one bond, fixed label shift:
// bra label = ket label + (dna, dnb).  Blocks (ket sector k, bra sector k'),
// row-major dim_k' x dim_k.
struct OpLayout {
  int dna = 0, dnb = 0;
  struct Blk { int ket, bra, rows, cols; size_t off; };
  std::vector<Blk> blk;
  std::vector<int> by_ket;  // ket sector -> block id or -1
  size_t size = 0;
};

inline void build_site_layout(SiteLayout& S, const Bond& bl, const Bond& br, int site, int width) {
  S.site = site;
  S.width = width;
  S.d = width == 1 ? 4 : 16;
  S.blk.clear();
  S.lookup.assign(bl.q.size() * S.d, -1);
  size_t off = 0;
  for (int a = 0; a < int(bl.q.size()); ++a)
    for (int n = 0; n < S.d; ++n) {
      QN dq = dot_qn(n, width);
      int c = br.find(QN{bl.q[a].na + dq.na, bl.q[a].nb + dq.nb});
      if (c < 0) continue;
      S.lookup[size_t(a) * S.d + n] = int(S.blk.size());
      S.blk.push_back({a, n, c, bl.dim[a], br.dim[c], off});
      off += size_t(bl.dim[a]) * br.dim[c];
    }
  S.size = off;
}

inline void build_op_layout(OpLayout& O, const Bond& B, int dna, int dnb) {
  O.dna = dna;
  O.dnb = dnb;
  O.blk.clear();
  O.by_ket.assign(B.q.size(), -1);
  size_t off = 0;
  for (int k = 0; k < int(B.q.size()); ++k) {
    int k2 = B.find(QN{B.q[k].na + dna, B.q[k].nb + dnb});
    if (k2 < 0) continue;
    O.by_ket[k] = int(O.blk.size());
    O.blk.push_back({k, k2, B.dim[k2], B.dim[k], off});
    off += size_t(B.dim[k2]) * B.dim[k];
  }
  O.size = off;
}

}  // namespace dmrg
