// Normal / complementary operator channels of the ab initio Hamiltonian and
// the site tensors that connect them (host side).
//
// The paper writes the superblock Hamiltonian as H_0^L x h_i x H_0^R and
// states that "x" is the summation over complementary operators (Sec. III B,
// eq. hzero_sb / hleft_sb).  This file makes that summation explicit.
//
// For a cut at bond b (left block = spin-orbitals of sites < b, right block =
// the rest) every term of H = sum t_pq a+_p a_q + sum_{p<q,r<s} W_pqrs
// a+_p a+_q a_r a_s (spin-orbitals, W antisymmetrized) is split into its
// left and right operator strings and assigned to one "channel" w, so that
// H = sum_w Lop_b[w] Rop_b[w]:
//   ID_H : (1, H_R)             H_ID : (H_L, 1)
//   CRE_L(p), DES_L(p)          single normal op a+_p / a_p on the left, the
//                               complementary S-type sum on the right
//   T_CRE(q), T_DES(q)          three-index complementary sum on the left,
//                               single normal op a+_q / a_q on the right
//   AA(p<q), DD(p<q), AD(p,q)   normal pair on the left (a+a+, aa, a+a), the
//                               complementary P / Q sums on the right
//   PP(r<s), PPB(p<q), QQ(q,r)  complementary pair sums on the left, normal
//                               pair on the right (aa, a+a+, a+a)
// Pairs are normal on the left for bonds b <= switch and on the right after.
//
// The site tensor W_b (a "dot" of one or two sites) expresses the channels of
// bond b+width through those of bond b:
//   Lop_{b+width}[w'] = sum_w Lop_b[w] (x) W[w,w'],
//   Rop_b[w] = sum_w' W[w,w'] (x) Rop_{b+width}[w'],
// with W[w,w'] a linear combination of normal-ordered ladder strings on the
// dot.  Fermion signs follow the Jordan-Wigner order (site-major, alpha
// before beta); the parity strings of the blocks are applied where the
// operators act (see the contraction code).
#pragma once
#include <cstdint>
#include <string>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace dmrg {

enum ChType : int {
  CH_ID_H = 0, CH_H_ID = 1, CH_CRE_L = 2, CH_DES_L = 3, CH_T_CRE = 4, CH_T_DES = 5,
  CH_AA = 6, CH_DD = 7, CH_AD = 8, CH_PP = 9, CH_PPB = 10, CH_QQ = 11
};

inline uint64_t chan_key(int t, int p, int q) {
  return (uint64_t(t) << 32) | (uint64_t(p + 1) << 16) | uint64_t(q + 1);
}
inline int key_type(uint64_t k) { return int(k >> 32); }
inline int key_p(uint64_t k) { return int((k >> 16) & 0xffff) - 1; }
inline int key_q(uint64_t k) { return int(k & 0xffff) - 1; }

// one ladder operator: spin-orbital index m = 2*site + spin, cre = creator
struct Lad { int8_t cre; int16_t m; };

struct Term {
  double c;
  int n;        // 0, 2 or 4 operators, normal ordered, creators ascending, annihilators ascending
  Lad op[4];
  int smin, smax;  // site range touched
};

struct Channel {
  uint64_t key;
  int dna, dnb;   // change of (n_alpha, n_beta) of the LEFT operator
  int parity;     // parity of the channel's operators (0 even, 1 odd)
  bool compl_left;  // the left operator is the complementary (summed) side
};

struct BondChannels {
  int mode;  // 0: pairs normal on the left, 1: pairs normal on the right
  std::vector<Channel> ch;
  std::unordered_map<uint64_t, int> idx;
  int find(uint64_t k) const {
    auto it = idx.find(k);
    return it == idx.end() ? -1 : it->second;
  }
};

// A normal-ordered ladder string on a dot of `width` sites (2*width modes):
// bit j of cre_mask / des_mask = mode (first dot mode + j) present.
struct DotString {
  int cre_mask, des_mask;
  int parity;
  int dna, dnb;    // change of the dot's (n_alpha, n_beta)
  // nonzero matrix elements <bra|s|ket> on the dot basis (d = 4^width)
  std::vector<int> bra, ket;
  std::vector<double> val;
};

struct WEntry {
  int src, dst;   // channel indices at bond b and bond b+width
  int sid;        // dot string id
  double c;
};

struct SiteOp {
  int b, width, d;
  std::vector<WEntry> e;
};

class QCHamiltonian {
 public:
  QCHamiltonian(int L, const double* h, const double* eri, double ecore, double screen = 1e-14);
  int L() const { return L_; }
  int switch_bond() const { return switch_; }
  // Pair mode of the operator sets: left operators at bond b keep the pairs
  // normal up to the switch bond, right operators up to one bond later, so
  // that the left and right sets met by a one-site dot always share a mode
  // (the normal -> complementary conversion then happens only inside one
  // renormalization step per direction, never inside a one-site sigma).
  int mode_left(int b) const { return b <= switch_ ? 0 : 1; }
  int mode_right(int b) const { return b <= switch_ + 1 ? 0 : 1; }
  const BondChannels& channels(int b, int mode) const;
  const BondChannels& left_channels(int b) const { return channels(b, mode_left(b)); }
  const BondChannels& right_channels(int b) const { return channels(b, mode_right(b)); }
  // dot strings of a dot with `width` sites (id space shared by all bonds)
  const DotString& dot_string(int width, int sid) const { return strings_[width - 1][sid]; }
  int num_dot_strings(int width) const { return int(strings_[width - 1].size()); }
  // site tensor for the dot starting at site b with 1 or 2 sites, from the
  // channels of bond b in mode m0 to those of bond b+width in mode m1 (cached)
  const SiteOp& site_op(int b, int width, int m0, int m1);
  size_t num_terms() const { return terms_.size(); }
  double ecore() const { return ecore_; }

 private:
  int L_, switch_;
  double ecore_;
  std::vector<Term> terms_;
  std::vector<std::vector<int>> terms_on_site_;
  std::vector<BondChannels> bonds_[2];  // per pair mode (built where used)
  std::vector<DotString> strings_[2];
  std::unordered_map<int, int> string_index_[2];
  std::unordered_map<int64_t, SiteOp> cache_;
  std::mutex cache_mu_;  // site_op() may be called from several plan threads

  void build_terms(const double* h, const double* eri, double screen);
  void build_channels();
  void build_strings(int width);
  uint64_t classify(const Lad* ops, int n, int b, int mode, int* nleft) const;
  Channel describe(uint64_t key, int b) const;
  int string_id(int width, int cre_mask, int des_mask) const;
};

}  // namespace dmrg
