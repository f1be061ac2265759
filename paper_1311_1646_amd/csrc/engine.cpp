// Context, MPS storage, operator pools, renormalization and sigma planners.
//
// Every contraction is planned on the host as lists of block GEMMs and
// executed by the device kernels in kernels.hip; no arithmetic of the method
// runs on the host.
#include "engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <tuple>

namespace dmrg {

// ---------------------------------------------------------------- buffers

DBuf& DBuf::operator=(DBuf&& o) noexcept {
  if (this != &o) {
    release();
    p = o.p;
    bytes = o.bytes;
    owner = o.owner;
    o.p = nullptr;
    o.bytes = 0;
  }
  return *this;
}

void DBuf::alloc(Ctx* c, size_t nbytes) {
  release();
  owner = c;
  bytes = nbytes;
  p = nbytes ? c->dev_alloc(nbytes) : nullptr;
}

void DBuf::ensure(Ctx* c, size_t nbytes) {
  if (nbytes > bytes) alloc(c, nbytes + nbytes / 4);
}

void DBuf::release() {
  if (p && owner) owner->dev_free(p);
  p = nullptr;
  bytes = 0;
}

int OpPool::add(const OpLayout* lay) {
  auto key = std::make_pair(lay->dna, lay->dnb);
  auto it = class_of.find(key);
  int c;
  if (it == class_of.end()) {
    c = int(classes.size());
    class_of[key] = c;
    classes.emplace_back();
    classes.back().lay = lay;
  } else {
    c = it->second;
  }
  items.push_back({c, classes[c].nslots++});
  return int(items.size()) - 1;
}

void OpPool::allocate(Ctx* x) {
  for (auto& C : classes) C.data.alloc(x, size_t(C.nslots) * C.lay->size * sizeof(double));
}

// ---------------------------------------------------------------- execution lists

int GemmList::job(void* C, int ldc, int m, int n, int flags) {
  auto it = job_of.find(C);
  if (it != job_of.end()) return it->second;
  int j = int(jobs.size());
  jobs.push_back({C, ldc, m, n, 0, 0, flags, 0});
  per_job.emplace_back();
  job_of[C] = j;
  return j;
}

double GemmList::flops(int batch) const {
  double f = 0;
  for (size_t j = 0; j < jobs.size(); ++j)
    for (auto& c : per_job[j])
      if (!(c.flags & GC_A_IDENTITY)) f += 2.0 * jobs[j].m * jobs[j].n * c.k;
  return f * batch;
}

namespace {
template <class T>
void upload(Ctx& x, DBuf& buf, const std::vector<T>& v) {
  buf.alloc(&x, v.size() * sizeof(T));
  if (!v.empty()) DMRG_HIP(hipMemcpy(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}
}  // namespace

void GemmList::run(Ctx& x, int batch, long sA, long sB, long sC) {
  if (jobs.empty()) return;
  std::vector<GContrib> con;
  std::vector<GTile> tiles;
  for (size_t j = 0; j < jobs.size(); ++j) {
    jobs[j].c0 = int(con.size());
    con.insert(con.end(), per_job[j].begin(), per_job[j].end());
    jobs[j].c1 = int(con.size());
    const int tm = (jobs[j].m + 63) / 64, tn = (jobs[j].n + 63) / 64;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) tiles.push_back({int(j), a, b, 0});
  }
  DBuf dt, dj, dc;
  upload(x, dt, tiles);
  upload(x, dj, jobs);
  upload(x, dc, con);
  launch_grouped_gemm_f64(dt.as<GTile>(), int(tiles.size()), dj.as<GJob>(), dc.as<GContrib>(), batch, sA, sB, sC,
                          x.stream);
  DMRG_HIP(hipGetLastError());
  DMRG_HIP(hipStreamSynchronize(x.stream));
}

void LinComb::run(Ctx& x, int batch, long stride) {
  if (!t.empty()) {
    DBuf dt, ds;
    upload(x, dt, t);
    upload(x, ds, s);
    launch_lincomb_f64(dt.as<LCTarget>(), int(t.size()), ds.as<LCSource>(), max_size, batch, stride, x.stream);
    DMRG_HIP(hipGetLastError());
    DMRG_HIP(hipStreamSynchronize(x.stream));
  }
  if (!d.empty()) {
    DBuf dd;
    upload(x, dd, d);
    launch_diag_add_f64(dd.as<DiagAdd>(), int(d.size()), 0, x.stream);
    DMRG_HIP(hipGetLastError());
    DMRG_HIP(hipStreamSynchronize(x.stream));
  }
}

// ---------------------------------------------------------------- context

Ctx::Ctx(int L_, int na, int nb, const double* h, const double* eri, double ecore, int dev, void* s,
         const dmrg_allocator* alloc)
    : L(L_), Na(na), Nb(nb), device(dev) {
  DMRG_REQUIRE(L >= 2 && L <= 128, DMRG_ERR_INVALID_ARG, "L must be in [2, 128]");
  DMRG_REQUIRE(na >= 0 && nb >= 0 && na <= L && nb <= L, DMRG_ERR_INVALID_ARG, "electron counts out of range");
  DMRG_REQUIRE(h && eri, DMRG_ERR_INVALID_ARG, "null integrals");
  if (alloc) allocator = *alloc;
  stream = static_cast<hipStream_t>(s);
  if (device >= 0) DMRG_HIP(hipSetDevice(device));
  H.reset(new QCHamiltonian(L, h, eri, ecore));
}

Ctx::~Ctx() {
  left.clear();
  right.clear();
  site.clear();
}

void Ctx::require_gpu() const {
  DMRG_REQUIRE(device >= 0, DMRG_ERR_STATE, "host-only context: no device calls");
}

void* Ctx::dev_alloc(size_t bytes) {
  require_gpu();
  void* p = nullptr;
  if (allocator.alloc) {
    p = allocator.alloc(bytes, stream, allocator.user);
    DMRG_REQUIRE(p, DMRG_ERR_OOM, "allocator callback returned null");
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(DMRG_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void Ctx::dev_free(void* p) {
  if (!p) return;
  if (allocator.free) allocator.free(p, allocator.user);
  else (void)hipFree(p);
}

const SiteLayout& Ctx::layout(int i, int width) {
  DMRG_REQUIRE(have_mps, DMRG_ERR_STATE, "no MPS");
  DMRG_REQUIRE(i >= 0 && width >= 1 && width <= 2 && i + width <= L, DMRG_ERR_INVALID_ARG, "bad site/width");
  auto key = std::make_pair(i, width);
  auto it = layouts_.find(key);
  if (it != layouts_.end()) return *it->second;
  auto S = std::make_unique<SiteLayout>();
  build_site_layout(*S, bonds[i], bonds[i + width], i, width);
  return *(layouts_[key] = std::move(S));
}

const OpLayout* Ctx::op_layout(int bond, int dna, int dnb) {
  auto key = std::make_tuple(bond, dna, dnb);
  auto it = op_layouts_.find(key);
  if (it != op_layouts_.end()) return it->second.get();
  auto O = std::make_unique<OpLayout>();
  build_op_layout(*O, bonds[bond], dna, dnb);
  return (op_layouts_[key] = std::move(O)).get();
}

// ---------------------------------------------------------------- MPS import/export

void Ctx::import_mps(const int* nsec, const int* sectors, const double* Ld, const double* Rd, const double* Cd,
                     const double* lamd) {
  require_gpu();
  DMRG_REQUIRE(nsec && sectors && Ld && Rd && Cd && lamd, DMRG_ERR_INVALID_ARG, "null MPS arrays");
  std::vector<Bond> B(L + 1);
  int k = 0;
  for (int b = 0; b <= L; ++b) {
    DMRG_REQUIRE(nsec[b] >= 1, DMRG_ERR_INVALID_ARG, "empty bond");
    for (int s = 0; s < nsec[b]; ++s, ++k) {
      QN q{sectors[3 * k], sectors[3 * k + 1]};
      int d = sectors[3 * k + 2];
      DMRG_REQUIRE(d >= 1, DMRG_ERR_INVALID_ARG, "sector dimension < 1");
      DMRG_REQUIRE(B[b].q.empty() || B[b].q.back() < q, DMRG_ERR_INVALID_ARG, "sectors not sorted");
      B[b].idx[q.key()] = int(B[b].q.size());
      B[b].q.push_back(q);
      B[b].dim.push_back(d);
    }
  }
  DMRG_REQUIRE(B[0].q.size() == 1 && B[0].q[0] == (QN{0, 0}) && B[0].dim[0] == 1, DMRG_ERR_INVALID_ARG,
               "bond 0 must be the vacuum");
  DMRG_REQUIRE(B[L].q.size() == 1 && B[L].q[0] == (QN{Na, Nb}) && B[L].dim[0] == 1, DMRG_ERR_INVALID_ARG,
               "bond L must hold the target (n_alpha, n_beta)");
  bonds = std::move(B);
  layouts_.clear();
  op_layouts_.clear();
  left.clear();
  right.clear();
  have_mps = true;
  site.clear();
  site.resize(L);
  size_t off = 0;
  for (int i = 0; i < L; ++i) {
    const SiteLayout& S = layout(i, 1);
    for (auto* pr : {&site[i].L, &site[i].R, &site[i].C}) pr->alloc(this, std::max<size_t>(S.size, 1) * 8);
    DMRG_HIP(hipMemcpy(site[i].L.p, Ld + off, S.size * 8, hipMemcpyHostToDevice));
    DMRG_HIP(hipMemcpy(site[i].R.p, Rd + off, S.size * 8, hipMemcpyHostToDevice));
    DMRG_HIP(hipMemcpy(site[i].C.p, Cd + off, S.size * 8, hipMemcpyHostToDevice));
    off += S.size;
  }
  lam.assign(L + 1, {});
  size_t lo = 0;
  for (int b = 0; b <= L; ++b)
    for (size_t s = 0; s < bonds[b].q.size(); ++s) {
      lam[b].emplace_back(lamd + lo, lamd + lo + bonds[b].dim[s]);
      lo += bonds[b].dim[s];
    }
}

void Ctx::export_mps(int* nsec_out, int* sectors_out, double* Ld, double* Rd, double* Cd, double* lam_out,
                     size_t* sizes) {
  DMRG_REQUIRE(have_mps, DMRG_ERR_STATE, "no MPS");
  size_t ns = 0, nd = 0, nl = 0;
  for (int b = 0; b <= L; ++b) {
    if (nsec_out) nsec_out[b] = int(bonds[b].q.size());
    for (size_t s = 0; s < bonds[b].q.size(); ++s) {
      if (sectors_out) {
        sectors_out[3 * ns] = bonds[b].q[s].na;
        sectors_out[3 * ns + 1] = bonds[b].q[s].nb;
        sectors_out[3 * ns + 2] = bonds[b].dim[s];
      }
      if (lam_out) std::memcpy(lam_out + nl, lam[b][s].data(), lam[b][s].size() * 8);
      nl += bonds[b].dim[s];
      ++ns;
    }
  }
  for (int i = 0; i < L; ++i) {
    const SiteLayout& S = layout(i, 1);
    if (Ld) DMRG_HIP(hipMemcpy(Ld + nd, site[i].L.p, S.size * 8, hipMemcpyDeviceToHost));
    if (Rd) DMRG_HIP(hipMemcpy(Rd + nd, site[i].R.p, S.size * 8, hipMemcpyDeviceToHost));
    if (Cd) DMRG_HIP(hipMemcpy(Cd + nd, site[i].C.p, S.size * 8, hipMemcpyDeviceToHost));
    nd += S.size;
  }
  if (sizes) {
    sizes[0] = ns;
    sizes[1] = nd;
    sizes[2] = nd;
    sizes[3] = nl;
  }
}

// ---------------------------------------------------------------- operator sets

void Ctx::alloc_opset(OpSet& S, int bond, int side) {
  const BondChannels& B = H->channels(bond);
  S.bond = bond;
  S.side = side;
  S.classes.clear();
  S.cls.assign(B.ch.size(), -1);
  S.slot.assign(B.ch.size(), 0);
  std::map<std::pair<int, int>, int> cls_of;
  const uint64_t ident = side == 0 ? chan_key(CH_ID_H, -1, -1) : chan_key(CH_H_ID, -1, -1);
  for (size_t w = 0; w < B.ch.size(); ++w) {
    if (B.ch[w].key == ident) continue;
    auto key = std::make_pair(B.ch[w].dna, B.ch[w].dnb);
    auto it = cls_of.find(key);
    int c;
    if (it == cls_of.end()) {
      c = int(S.classes.size());
      cls_of[key] = c;
      S.classes.emplace_back();
      S.classes.back().lay = op_layout(bond, key.first, key.second);
    } else {
      c = it->second;
    }
    S.cls[w] = c;
    S.slot[w] = S.classes[c].nslots++;
  }
  for (auto& C : S.classes) C.data.alloc(this, std::max<size_t>(size_t(C.nslots) * C.lay->size, 1) * 8);
  S.valid = true;
}


// ---------------------------------------------------------------- planning helpers

namespace {

struct Group {
  int key_ch;  // channel the group is keyed on
  int sid;     // dot string
  std::vector<std::pair<int, double>> src;  // (other channel, coefficient)
};

// Group the entries of W by (dst, sid) (by_dst) or by (src, sid).
std::vector<Group> group_entries(const SiteOp& W, bool by_dst, int skip_ch) {
  std::map<std::pair<int, int>, int> gi;
  std::vector<Group> G;
  for (const WEntry& e : W.e) {
    const int k = by_dst ? e.dst : e.src;
    const int o = by_dst ? e.src : e.dst;
    if (k == skip_ch) continue;
    auto key = std::make_pair(k, e.sid);
    auto it = gi.find(key);
    int g;
    if (it == gi.end()) {
      g = int(G.size());
      gi[key] = g;
      G.push_back({k, e.sid, {}});
    } else {
      g = it->second;
    }
    G[g].src.push_back({o, e.c});
  }
  return G;
}

inline int opblk(const ORef& r, int ket) { return r.identity() ? ket : r.lay->by_ket[ket]; }
inline int opbra(const ORef& r, int ket) {
  if (r.identity()) return ket;
  const int b = r.lay->by_ket[ket];
  return b < 0 ? -1 : r.lay->blk[b].bra;
}
inline const double* opptr(const ORef& r, int ket) { return r.p + r.lay->blk[r.lay->by_ket[ket]].off; }

using Sources = std::vector<std::pair<ORef, double>>;

// Renormalization job: target += alpha * R(X, sid), R the one-site transform.
struct RJob {
  ORef X;
  int dressed;  // >= 0: X is this dressed-pool item (resolved after allocation)
  double alpha;
  int sid;
  int tkind;    // 0: channel of the destination set, 1: building-block item
  int tgt;
  int pz;       // parity of the right-block operator (right renormalization sign)
};

struct DressPlan {
  OpPool dressed, blocks;
  std::vector<std::pair<int, Sources>> pend;
  std::vector<RJob> jobs;
  std::vector<std::tuple<int, int, double>> combine;  // (target channel, block item, c)
};

// Form all pending dressed operators: out = sum c_j src_j (+ c_id * 1).
void emit_dressed(OpPool& pool, const std::vector<std::pair<int, Sources>>& pend, LinComb& lc) {
  for (auto& pr : pend) {
    ORef out = pool.ref(pr.first);
    lc.target(const_cast<double*>(out.p), long(out.lay->size), false);
    double cid = 0.0;
    for (auto& s : pr.second) {
      if (s.first.identity()) cid += s.second;
      else lc.source(s.first.p, s.second);
    }
    if (cid != 0.0) {
      DMRG_REQUIRE(out.lay->dna == 0 && out.lay->dnb == 0, DMRG_ERR_INTERNAL, "identity in a shifted class");
      for (auto& b : out.lay->blk)
        if (b.ket == b.bra) lc.d.push_back({const_cast<double*>(out.p) + b.off, b.rows, 0, cid});
    }
  }
}

}  // namespace

// Decide, per target group, whether the sources are combined before the
// one-site transform (one dressed operator per target) or after it (one
// transformed building block per shared source, then a linear combination):
// the cheaper one by the number of transforms each target accounts for.
static void plan_renorm(Ctx& x, const std::vector<Group>& G, const OpSet& src, const BondChannels& Bt,
                        const BondChannels& Bs, int dressed_bond, int target_bond, bool left, DressPlan& P) {
  std::map<std::pair<int, int>, int> fan;
  for (auto& g : G)
    for (auto& s : g.src) fan[{s.first, g.sid}]++;
  P.dressed.bond = dressed_bond;
  P.blocks.bond = target_bond;
  std::map<std::pair<int, int>, int> block_of;
  for (auto& g : G) {
    double share = 0;
    for (auto& s : g.src) share += 1.0 / fan[{s.first, g.sid}];
    const bool after = g.src.size() > 1 && share < 1.0 - 1e-9;
    const DotString& ds = x.H->dot_string(1, g.sid);
    const Channel& tch = Bt.ch[g.key_ch];
    const int pz = left ? 0 : Bs.ch[g.src[0].first].parity;
    if (!after) {
      if (g.src.size() == 1) {
        P.jobs.push_back({src.ref(g.src[0].first), -1, g.src[0].second, g.sid, 0, g.key_ch, pz});
      } else {
        Sources ss;
        for (auto& s : g.src) ss.push_back({src.ref(s.first), s.second});
        const int sa = left ? tch.dna - ds.dna : tch.dna + ds.dna;
        const int sb = left ? tch.dnb - ds.dnb : tch.dnb + ds.dnb;
        const int id = P.dressed.add(x.op_layout(dressed_bond, sa, sb));
        P.pend.push_back({id, std::move(ss)});
        P.jobs.push_back({ORef{}, id, 1.0, g.sid, 0, g.key_ch, pz});
      }
    } else {
      for (auto& s : g.src) {
        auto key = std::make_pair(s.first, g.sid);
        auto it = block_of.find(key);
        int item;
        if (it == block_of.end()) {
          item = P.blocks.add(x.op_layout(target_bond, tch.dna, tch.dnb));
          block_of[key] = item;
          const int pzs = left ? 0 : Bs.ch[s.first].parity;
          P.jobs.push_back({src.ref(s.first), -1, 1.0, g.sid, 1, item, pzs});
        } else {
          item = it->second;
        }
        P.combine.push_back({g.key_ch, item, s.second});
      }
    }
  }
  P.dressed.allocate(&x);
  P.blocks.allocate(&x);
  for (auto& j : P.jobs)
    if (j.dressed >= 0) j.X = P.dressed.ref(j.dressed);
}

static void finish_renorm(Ctx& x, DressPlan& P, OpSet& dst) {
  LinComb post;
  std::map<int, std::vector<std::pair<int, double>>> by_tgt;
  for (auto& cb : P.combine) by_tgt[std::get<0>(cb)].push_back({std::get<1>(cb), std::get<2>(cb)});
  for (auto& kv : by_tgt) {
    ORef t = dst.ref(kv.first);
    post.target(const_cast<double*>(t.p), long(t.lay->size), true);
    for (auto& s : kv.second) post.source(P.blocks.ref(s.first).p, s.second);
  }
  post.run(x, 1, 0);
}

// ---------------------------------------------------------------- renormalization

// Left block, across site i (bond i -> i+1):
// Lop_{i+1}[w'] = sum_{(w,sid)} c A_bra^T (Lop_i[w] P^{p(sid)} (x) sid) A_ket.
void Ctx::renorm_left(int i, const double* Abra, const double* Aket, const OpSet& src, OpSet& dst) {
  const SiteOp& W = H->site_op(i, 1);
  const SiteLayout& S = layout(i, 1);
  const Bond& bl = bonds[i];
  const BondChannels& B1 = H->channels(i + 1);
  std::vector<Group> G = group_entries(W, true, B1.find(chan_key(CH_ID_H, -1, -1)));
  DressPlan P;
  plan_renorm(*this, G, src, B1, H->channels(i), i, i + 1, true, P);
  for (auto& C : dst.classes) launch_fill_f64(C.data.as<double>(), long(C.data.bytes / 8), 0.0, stream);
  for (auto& C : P.blocks.classes) launch_fill_f64(C.data.as<double>(), long(C.data.bytes / 8), 0.0, stream);
  LinComb form;
  emit_dressed(P.dressed, P.pend, form);
  form.run(*this, 1, 0);
  // stage 1: T(X, a, n) = X(a'<-a) A_ket(a, n, c)
  GemmList st1, st2;
  std::map<std::pair<const double*, int>, size_t> toff;
  size_t tsize = 0;
  std::vector<std::tuple<ORef, int, size_t>> need;
  for (auto& j : P.jobs) {
    if (j.X.identity()) continue;
    const DotString& ds = H->dot_string(1, j.sid);
    for (size_t e = 0; e < ds.val.size(); ++e)
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, ds.ket[e]);
        if (b < 0 || opblk(j.X, a) < 0) continue;
        auto key = std::make_pair(j.X.p, b);
        if (toff.count(key)) continue;
        toff[key] = tsize;
        need.push_back({j.X, b, tsize});
        tsize += size_t(bl.dim[opbra(j.X, a)]) * S.blk[b].cols;
      }
  }
  DBuf T;
  T.alloc(this, std::max<size_t>(tsize, 1) * 8);
  double* Tp = T.as<double>();
  for (auto& nd : need) {
    const ORef& X = std::get<0>(nd);
    const auto& blk = S.blk[std::get<1>(nd)];
    const int ap = opbra(X, blk.a);
    const int jb = st1.job(Tp + std::get<2>(nd), blk.cols, bl.dim[ap], blk.cols, 0);
    st1.add(jb, {opptr(X, blk.a), Aket + blk.off, blk.rows, blk.cols, blk.rows, 0, 1.0});
  }
  // stage 2: target(c'<-c) += alpha val sign A_bra(a',n',c')^T T
  for (auto& j : P.jobs) {
    const DotString& ds = H->dot_string(1, j.sid);
    const ORef tgt = j.tkind == 0 ? dst.ref(j.tgt) : P.blocks.ref(j.tgt);
    for (size_t e = 0; e < ds.val.size(); ++e)
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, ds.ket[e]);
        if (b < 0 || opblk(j.X, a) < 0) continue;
        const int ap = opbra(j.X, a);
        const int bp = S.find(ap, ds.bra[e]);
        if (bp < 0) continue;
        const int c = S.blk[b].c, cp = S.blk[bp].c;
        const int tb = tgt.lay->by_ket[c];
        DMRG_REQUIRE(tb >= 0 && tgt.lay->blk[tb].bra == cp, DMRG_ERR_INTERNAL, "left renorm target block mismatch");
        const double sign = (ds.parity && (bl.q[a].n() & 1)) ? -1.0 : 1.0;
        double* out = const_cast<double*>(tgt.p) + tgt.lay->blk[tb].off;
        const int jb = st2.job(out, S.blk[b].cols, S.blk[bp].cols, S.blk[b].cols, GJ_ACCUMULATE);
        const double* Bp = j.X.identity() ? Aket + S.blk[b].off : Tp + toff[{j.X.p, b}];
        st2.add(jb, {Abra + S.blk[bp].off, Bp, S.blk[bp].cols, S.blk[b].cols, bl.dim[ap], GC_TRANS_A,
                     j.alpha * ds.val[e] * sign});
      }
  }
  st1.run(*this, 1, 0, 0, 0);
  st2.run(*this, 1, 0, 0, 0);
  stats.renorm_flops += st1.flops(1) + st2.flops(1);
  finish_renorm(*this, P, dst);
}

// Right block, across site i (bond i+1 -> i):
// Rop_i[w] = sum_{(w',sid)} c R_bra (sid P_D^{p(w')} (x) Rop_{i+1}[w']) R_ket^T.
void Ctx::renorm_right(int i, const double* Abra, const double* Aket, const OpSet& src, OpSet& dst) {
  const SiteOp& W = H->site_op(i, 1);
  const SiteLayout& S = layout(i, 1);
  const Bond& bl = bonds[i];
  const Bond& br = bonds[i + 1];
  const BondChannels& B0 = H->channels(i);
  std::vector<Group> G = group_entries(W, false, B0.find(chan_key(CH_H_ID, -1, -1)));
  DressPlan P;
  plan_renorm(*this, G, src, B0, H->channels(i + 1), i + 1, i, false, P);
  for (auto& C : dst.classes) launch_fill_f64(C.data.as<double>(), long(C.data.bytes / 8), 0.0, stream);
  for (auto& C : P.blocks.classes) launch_fill_f64(C.data.as<double>(), long(C.data.bytes / 8), 0.0, stream);
  LinComb form;
  emit_dressed(P.dressed, P.pend, form);
  form.run(*this, 1, 0);
  // stage 1: T(Z, a, n) = Z(c'<-c) R_ket(a, n, c)^T   (m_c' x m_a)
  GemmList st1, st2;
  std::map<std::pair<const double*, int>, size_t> toff;
  size_t tsize = 0;
  std::vector<std::tuple<ORef, int, size_t>> need;
  for (auto& j : P.jobs) {
    if (j.X.identity()) continue;
    const DotString& ds = H->dot_string(1, j.sid);
    for (size_t e = 0; e < ds.val.size(); ++e)
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, ds.ket[e]);
        if (b < 0 || opblk(j.X, S.blk[b].c) < 0) continue;
        auto key = std::make_pair(j.X.p, b);
        if (toff.count(key)) continue;
        toff[key] = tsize;
        need.push_back({j.X, b, tsize});
        tsize += size_t(br.dim[opbra(j.X, S.blk[b].c)]) * S.blk[b].rows;
      }
  }
  DBuf T;
  T.alloc(this, std::max<size_t>(tsize, 1) * 8);
  double* Tp = T.as<double>();
  for (auto& nd : need) {
    const ORef& Z = std::get<0>(nd);
    const auto& blk = S.blk[std::get<1>(nd)];
    const int cp = opbra(Z, blk.c);
    const int jb = st1.job(Tp + std::get<2>(nd), blk.rows, br.dim[cp], blk.rows, 0);
    st1.add(jb, {opptr(Z, blk.c), Aket + blk.off, blk.cols, blk.cols, blk.cols, GC_TRANS_B, 1.0});
  }
  // stage 2: target(a'<-a) += alpha val sign R_bra(a',n',c') T
  for (auto& j : P.jobs) {
    const DotString& ds = H->dot_string(1, j.sid);
    const ORef tgt = j.tkind == 0 ? dst.ref(j.tgt) : P.blocks.ref(j.tgt);
    for (size_t e = 0; e < ds.val.size(); ++e) {
      const int n = ds.ket[e], np = ds.bra[e];
      const QN qn = site_qn(n), qnp = site_qn(np);
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, n);
        if (b < 0) continue;
        const int c = S.blk[b].c;
        if (opblk(j.X, c) < 0) continue;
        const int cp = opbra(j.X, c);
        const int ap = bl.find(QN{br.q[cp].na - qnp.na, br.q[cp].nb - qnp.nb});
        if (ap < 0) continue;
        const int bp = S.find(ap, np);
        if (bp < 0 || S.blk[bp].c != cp) continue;
        const int tb = tgt.lay->by_ket[a];
        DMRG_REQUIRE(tb >= 0 && tgt.lay->blk[tb].bra == ap, DMRG_ERR_INTERNAL, "right renorm target block mismatch");
        const double sign = (j.pz && ((qn.na + qn.nb) & 1)) ? -1.0 : 1.0;
        double* out = const_cast<double*>(tgt.p) + tgt.lay->blk[tb].off;
        const int jb = st2.job(out, S.blk[b].rows, S.blk[bp].rows, S.blk[b].rows, GJ_ACCUMULATE);
        const double al = j.alpha * ds.val[e] * sign;
        if (j.X.identity())
          st2.add(jb, {Abra + S.blk[bp].off, Aket + S.blk[b].off, S.blk[bp].cols, S.blk[b].cols, S.blk[b].cols,
                       GC_TRANS_B, al});
        else
          st2.add(jb, {Abra + S.blk[bp].off, Tp + toff[{j.X.p, b}], S.blk[bp].cols, S.blk[b].rows, br.dim[cp], 0, al});
      }
    }
  }
  st1.run(*this, 1, 0, 0, 0);
  st2.run(*this, 1, 0, 0, 0);
  stats.renorm_flops += st1.flops(1) + st2.flops(1);
  finish_renorm(*this, P, dst);
}

void Ctx::build_ops(int prec) {
  require_gpu();
  DMRG_REQUIRE(have_mps, DMRG_ERR_STATE, "import or compute an MPS first");
  DMRG_REQUIRE(prec == DMRG_FP64, DMRG_ERR_INVALID_ARG, "operator pools: only FP64 is built in this version");
  left.clear();
  right.clear();
  left.resize(L + 1);
  right.resize(L + 1);
  stats.renorm_flops = 0;
  hipEvent_t e0, e1;
  DMRG_HIP(hipEventCreate(&e0));
  DMRG_HIP(hipEventCreate(&e1));
  DMRG_HIP(hipEventRecord(e0, stream));
  alloc_opset(left[0], 0, 0);
  for (int i = 0; i < L; ++i) {
    alloc_opset(left[i + 1], i + 1, 0);
    renorm_left(i, site[i].L.as<double>(), site[i].L.as<double>(), left[i], left[i + 1]);
  }
  alloc_opset(right[L], L, 1);
  for (int i = L - 1; i >= 0; --i) {
    alloc_opset(right[i], i, 1);
    renorm_right(i, site[i].R.as<double>(), site[i].R.as<double>(), right[i + 1], right[i]);
  }
  DMRG_HIP(hipEventRecord(e1, stream));
  DMRG_HIP(hipEventSynchronize(e1));
  float ms = 0;
  DMRG_HIP(hipEventElapsedTime(&ms, e0, e1));
  stats.renorm_ms = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  double b = 0;
  for (auto& s : left) b += double(s.bytes());
  for (auto& s : right) b += double(s.bytes());
  stats.op_bytes = b;
  ops_prec = prec;
}

// ---------------------------------------------------------------- sigma

namespace {
struct STerm {
  ORef X, Z;
  int sid;
  double alpha;
  int pz;  // parity of the right-block operator
};
}  // namespace

// sigma = sum_t alpha_t (X_t P^{p(sid)+p(Z)} (x) sid P_D^{p(Z)} (x) Z_t) C
static void exec_sigma(Ctx& x, int i, int width, const std::vector<STerm>& terms, int nvec, const double* Cin,
                       double* Sout, double* flops_out, float* ms_out, float* main_ms) {
  const SiteLayout& S = x.layout(i, width);
  const Bond& bl = x.bonds[i];
  const Bond& br = x.bonds[i + width];
  GemmList st1, st2;
  std::map<std::pair<const double*, int>, size_t> toff;
  size_t tsize = 0;
  std::vector<std::tuple<ORef, int, size_t>> need;
  for (auto& t : terms) {
    if (t.Z.identity()) continue;
    const DotString& ds = x.H->dot_string(width, t.sid);
    for (size_t e = 0; e < ds.val.size(); ++e)
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, ds.ket[e]);
        if (b < 0 || opblk(t.Z, S.blk[b].c) < 0 || opblk(t.X, a) < 0) continue;
        auto key = std::make_pair(t.Z.p, b);
        if (toff.count(key)) continue;
        toff[key] = tsize;
        need.push_back({t.Z, b, tsize});
        tsize += size_t(S.blk[b].rows) * br.dim[opbra(t.Z, S.blk[b].c)];
      }
  }
  DBuf T;
  T.alloc(&x, std::max<size_t>(tsize, 1) * 8 * nvec);
  double* Tp = T.as<double>();
  // stage 1: T(Z, a, n, c) = C(a,n,c) Z(c'<-c)^T   (m_a x m_c')
  for (auto& nd : need) {
    const ORef& Z = std::get<0>(nd);
    const auto& blk = S.blk[std::get<1>(nd)];
    const int cp = opbra(Z, blk.c);
    const int jb = st1.job(Tp + std::get<2>(nd), br.dim[cp], blk.rows, br.dim[cp], GJ_C_BATCHED);
    st1.add(jb, {Cin + blk.off, opptr(Z, blk.c), blk.cols, blk.cols, blk.cols, GC_TRANS_B | GC_A_BATCHED, 1.0});
  }
  // stage 2: sigma(a',n',c') = sum alpha val sign X(a'<-a) T
  for (size_t b = 0; b < S.blk.size(); ++b)
    st2.job(Sout + S.blk[b].off, S.blk[b].cols, S.blk[b].rows, S.blk[b].cols, GJ_C_BATCHED);
  for (auto& t : terms) {
    const DotString& ds = x.H->dot_string(width, t.sid);
    for (size_t e = 0; e < ds.val.size(); ++e) {
      const int n = ds.ket[e], np = ds.bra[e];
      const int nd = dot_qn(n, width).n();
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, n);
        if (b < 0) continue;
        const int c = S.blk[b].c;
        if (opblk(t.Z, c) < 0 || opblk(t.X, a) < 0) continue;
        const int cp = opbra(t.Z, c), ap = opbra(t.X, a);
        const int bp = S.find(ap, np);
        if (bp < 0 || S.blk[bp].c != cp) continue;
        int sgn = 1;
        if (((ds.parity + t.pz) & 1) && (bl.q[a].n() & 1)) sgn = -sgn;
        if (t.pz && (nd & 1)) sgn = -sgn;
        const int jb = st2.job(Sout + S.blk[bp].off, S.blk[bp].cols, S.blk[bp].rows, S.blk[bp].cols, GJ_C_BATCHED);
        GContrib g;
        g.A = t.X.identity() ? nullptr : opptr(t.X, a);
        g.lda = S.blk[b].rows;
        g.k = S.blk[b].rows;
        g.alpha = t.alpha * ds.val[e] * sgn;
        g.flags = (t.X.identity() ? GC_A_IDENTITY : 0);
        if (t.Z.identity()) {
          g.B = Cin + S.blk[b].off;
          g.ldb = S.blk[b].cols;
          g.flags |= GC_B_BATCHED_ALT;
        } else {
          g.flags |= GC_B_BATCHED;
          g.B = Tp + toff[{t.Z.p, b}];
          g.ldb = br.dim[cp];
        }
        st2.add(jb, g);
      }
    }
  }
  hipEvent_t e0, e1, e2;
  DMRG_HIP(hipEventCreate(&e0));
  DMRG_HIP(hipEventCreate(&e1));
  DMRG_HIP(hipEventCreate(&e2));
  DMRG_HIP(hipEventRecord(e0, x.stream));
  st1.run(x, nvec, long(S.size), 0, long(tsize));
  DMRG_HIP(hipEventRecord(e1, x.stream));
  st2.run(x, nvec, long(S.size), long(tsize), long(S.size));
  DMRG_HIP(hipEventRecord(e2, x.stream));
  DMRG_HIP(hipEventSynchronize(e2));
  float a = 0, b2 = 0;
  DMRG_HIP(hipEventElapsedTime(&a, e0, e2));
  DMRG_HIP(hipEventElapsedTime(&b2, e1, e2));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  if (flops_out) {
    flops_out[0] = st1.flops(nvec) + st2.flops(nvec);
    flops_out[1] = st2.flops(nvec);
  }
  if (ms_out) *ms_out = a;
  if (main_ms) *main_ms = b2;
}

// Terms of the effective Hamiltonian on the dot (i, width): the channel site
// operator is dressed on the side that needs fewer formed operators.
static std::vector<STerm> sigma_terms(Ctx& x, int i, int width, OpPool& pool, LinComb& form) {
  const SiteOp& W = x.H->site_op(i, width);
  const OpSet& Lset = x.left[i];
  const OpSet& Rset = x.right[i + width];
  const BondChannels& B0 = x.H->channels(i);
  const BondChannels& B1 = x.H->channels(i + width);
  std::vector<Group> GL = group_entries(W, true, -1), GR = group_entries(W, false, -1);
  size_t fl = 0, fr = 0;
  for (auto& g : GL) fl += g.src.size() > 1;
  for (auto& g : GR) fr += g.src.size() > 1;
  const bool left_dressed = fl <= fr;
  std::vector<STerm> terms;
  std::vector<std::pair<int, Sources>> pend;
  std::vector<std::pair<size_t, int>> fix;  // term -> dressed item
  pool.bond = left_dressed ? i : i + width;
  for (auto& g : left_dressed ? GL : GR) {
    const DotString& ds = x.H->dot_string(width, g.sid);
    STerm t{};
    t.sid = g.sid;
    if (left_dressed) {
      t.Z = Rset.ref(g.key_ch);
      t.pz = B1.ch[g.key_ch].parity;
      if (g.src.size() == 1) {
        t.X = Lset.ref(g.src[0].first);
        t.alpha = g.src[0].second;
      } else {
        Sources ss;
        for (auto& s : g.src) ss.push_back({Lset.ref(s.first), s.second});
        const Channel& ch = B1.ch[g.key_ch];
        const int id = pool.add(x.op_layout(i, ch.dna - ds.dna, ch.dnb - ds.dnb));
        pend.push_back({id, std::move(ss)});
        fix.push_back({terms.size(), id});
        t.alpha = 1.0;
      }
    } else {
      t.X = Lset.ref(g.key_ch);
      t.pz = B1.ch[g.src[0].first].parity;
      if (g.src.size() == 1) {
        t.Z = Rset.ref(g.src[0].first);
        t.alpha = g.src[0].second;
      } else {
        Sources ss;
        for (auto& s : g.src) ss.push_back({Rset.ref(s.first), s.second});
        const Channel& ch = B0.ch[g.key_ch];
        const int id = pool.add(x.op_layout(i + width, ch.dna + ds.dna, ch.dnb + ds.dnb));
        pend.push_back({id, std::move(ss)});
        fix.push_back({terms.size(), id});
        t.alpha = 1.0;
      }
    }
    terms.push_back(t);
  }
  pool.allocate(&x);
  for (auto& f : fix) {
    if (left_dressed) terms[f.first].X = pool.ref(f.second);
    else terms[f.first].Z = pool.ref(f.second);
  }
  emit_dressed(pool, pend, form);
  return terms;
}

void Ctx::sigma(int i, int width, int nvec, const double* Cin, double* Sout) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(nvec >= 1 && Cin && Sout, DMRG_ERR_INVALID_ARG, "bad sigma arguments");
  OpPool pool;
  LinComb form;
  std::vector<STerm> terms = sigma_terms(*this, i, width, pool, form);
  form.run(*this, 1, 0);
  double fl[2] = {0, 0};
  float ms = 0, mms = 0;
  exec_sigma(*this, i, width, terms, nvec, Cin, Sout, fl, &ms, &mms);
  stats.sigma_flops = fl[0];
  stats.sigma_main_flops = fl[1];
  stats.sigma_ms = ms;
  stats.sigma_main_ms = mms;
}

void Ctx::diag(int i, int width, double* out) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  OpPool pool;
  LinComb form;
  std::vector<STerm> terms = sigma_terms(*this, i, width, pool, form);
  form.run(*this, 1, 0);
  const SiteLayout& S = layout(i, width);
  const Bond& bl = bonds[i];
  std::vector<std::vector<DiagTerm>> per(S.blk.size());
  for (auto& t : terms) {
    if (t.X.lay && (t.X.lay->dna || t.X.lay->dnb)) continue;
    if (t.Z.lay && (t.Z.lay->dna || t.Z.lay->dnb)) continue;
    const DotString& ds = H->dot_string(width, t.sid);
    for (size_t e = 0; e < ds.val.size(); ++e) {
      if (ds.bra[e] != ds.ket[e]) continue;
      const int n = ds.ket[e];
      const int nd = dot_qn(n, width).n();
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, n);
        if (b < 0) continue;
        const int c = S.blk[b].c;
        if (opblk(t.X, a) < 0 || opblk(t.Z, c) < 0) continue;
        int sgn = 1;
        if (((ds.parity + t.pz) & 1) && (bl.q[a].n() & 1)) sgn = -sgn;
        if (t.pz && (nd & 1)) sgn = -sgn;
        per[b].push_back({t.X.identity() ? nullptr : opptr(t.X, a), t.Z.identity() ? nullptr : opptr(t.Z, c),
                          t.alpha * ds.val[e] * sgn});
      }
    }
  }
  std::vector<DiagJob> jobs;
  std::vector<DiagTerm> dt;
  for (size_t b = 0; b < S.blk.size(); ++b) {
    jobs.push_back({out + S.blk[b].off, S.blk[b].rows, S.blk[b].cols, int(dt.size()), 0});
    dt.insert(dt.end(), per[b].begin(), per[b].end());
    jobs.back().t1 = int(dt.size());
  }
  DBuf dj, dd;
  upload(*this, dj, jobs);
  upload(*this, dd, dt);
  launch_diag_jobs_f64(dj.as<DiagJob>(), int(jobs.size()), dd.as<DiagTerm>(), stream);
  DMRG_HIP(hipGetLastError());
  DMRG_HIP(hipStreamSynchronize(stream));
}

}  // namespace dmrg
