// Context, MPS storage, operator sets, and the planners of the block
// renormalization and of the sigma vector.
//
// Every contraction is planned once on the host as device-resident lists of
// block GEMMs addressed relative to base slots, and executed by the kernels
// in kernels.hip; no arithmetic of the method runs on the host.
#include "engine.hpp"
#include "kernels_mfma.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <set>
#include <unordered_map>

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
  if (nbytes > bytes) {
    if (p) c->sync();  // work still queued may use the old buffer
    release();
    alloc(c, nbytes + nbytes / 8);
  }
}

void DBuf::release() {
  if (p && owner) owner->dev_free(p);
  p = nullptr;
  bytes = 0;
}

namespace {
template <class T>
void upload(Ctx& x, DBuf& buf, const std::vector<T>& v) {
  buf.alloc(&x, v.size() * sizeof(T));
  if (!v.empty()) DMRG_HIP(hipMemcpy(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}
}  // namespace

void GemmPlan::launch(Ctx& x, const Bases& b, int batch, int prec, bool out_f64, const Bases* bout,
                      int role) const {
  if (ntiles == 0) return;
  if (prec == DMRG_FP64 && !x.fp64_mfma) {
    if (role == 1) x.mark_main(true);
    launch_grouped_gemm_f64(tiles.as<GTile>(), ntiles, jobs.as<GJob>(), con.as<GContrib>(), gat.as<int>(), b, batch,
                            x.stream);
    if (role == 1) x.mark_main(false);
    DMRG_HIP(hipGetLastError());
    return;
  }
  const Bases& bo = bout ? *bout : b;
  auto batched = [](const Bases& q, unsigned mask, bool all) {
    bool any = false, every = true;
    for (int k = 0; k < kMaxBases; ++k)
      if (mask >> k & 1u) {
        any |= q.stride[k] != 0;
        every &= q.stride[k] != 0;
      }
    return all ? (every && mask != 0) : any;
  };
  int fold = FOLD_NONE;
  if (batch > 1 && batched(bo, mask_c, true)) {
    if (!batched(b, mask_a, false) && batched(b, mask_b, true)) fold = FOLD_N;
    else if (!batched(b, mask_b, false) && (mask_a == 0 || batched(b, mask_a, true))) fold = FOLD_M;
  }
  // 128x128 tiles exist for FP32 operands only (FP32, BF16x3)
  int want = x.tile_policy[prec][role == 1 ? 1 : 0][fold];
  if (prec == DMRG_FP64 && want == TILE_128x128) want = TILE_64x64;
  if (want < 0 && prec != DMRG_FP64)
    if (const char* e = std::getenv("DMRG_TILE_SHAPE"))
      if (std::string(e) == "128x128") want = TILE_128x128;
  const FoldTiles& F = fold_lists(x, fold, batch, want);
  void* part = nullptr;
  if (F.nslots > 0) {
    const size_t esz = prec == DMRG_FP64 ? 8 : 4;
    const size_t tile = size_t(tile_rows(F.shape)) * tile_cols(F.shape);
    part = x.workspace(WS_PART, x.ws_part, size_t(F.nslots) * (fold == FOLD_NONE ? batch : 1) * tile * esz);
  }
  if (role == 1) x.mark_main(true);
  launch_grouped_gemm(prec, out_f64, role, F.shape, F.tiles.as<GTile>(), F.ntiles, jobs.as<GJob>(),
                      con.as<GContrib>(), gat.as<int>(), F.segs.as<GSeg>(), F.nslots, part, b, bo, fold, batch, x.stream);
  if (role == 1) x.mark_main(false);
  launch_reduce_partials(prec, out_f64, F.shape, F.red.as<GRed>(), F.nred, jobs.as<GJob>(), F.nslots, part, bo, fold,
                         batch, x.stream);
  DMRG_HIP(hipGetLastError());
}

// Tiles of every job for this fold and batch; the contribution list of a
// job whose work is far above the average share of a workgroup is split into
// segments (one tile per segment, partial sums reduced afterwards), so that
// a few long jobs do not leave the rest of the chip idle.
const GemmPlan::FoldTiles& GemmPlan::fold_lists(Ctx& x, int fold, int batch, int want) const {
  // an explicit shape (autotuner) may put 128 along either dimension; the
  // planner's own choice below puts it only along the unfolded one
  const auto key = std::make_tuple(fold, batch, want);
  FoldTiles& F = fold_tiles[key];
  if (F.ntiles > 0) return F;
  const long entries = fold == FOLD_NONE ? batch : 1;
  std::vector<long> tiles_of(shapes.size()), work_of(shapes.size());
  for (size_t j = 0; j < shapes.size(); ++j) {
    long w = 0;
    for (int c = ranges[j].first; c < ranges[j].second; ++c) w += (con_k[c] + 31) / 32;
    work_of[j] = w;
  }
  // Tile shape: 128 along the unfolded (block) dimension only when it pads
  // much less than 64-wide tiles (the wider tiles hold more LDS and
  // registers, so fewer workgroups are resident; measured slower at equal
  // padding).
  auto padded = [&](int sh) {
    const long tr = tile_rows(sh), tc = tile_cols(sh);
    double w = 0;
    for (size_t j = 0; j < shapes.size(); ++j) {
      const long m = fold == FOLD_M ? long(shapes[j].first) * batch : shapes[j].first;
      const long n = fold == FOLD_N ? long(shapes[j].second) * batch : shapes[j].second;
      w += double((m + tr - 1) / tr * tr) * double((n + tc - 1) / tc * tc) * double(work_of[j]);
    }
    return sh == TILE_64x64 ? w : 1.5 * w;  // the wider tiles run at lower occupancy
  };
  int shape = TILE_64x64;
  if (want >= 0) {
    shape = want;  // set by the autotuner (Ctx::autotune)
  } else {
    double best = padded(TILE_64x64);
    for (int sh : {TILE_128x64, TILE_64x128}) {
      if ((fold == FOLD_N && sh == TILE_64x128) || (fold == FOLD_M && sh == TILE_128x64)) continue;
      const double c = padded(sh);
      if (c < best) {
        best = c;
        shape = sh;
      }
    }
    // DMRG_TILE_SHAPE=64x64|128x64|64x128 fixes the shape of every launch
    // (128x128, FP32 operands only, is applied by the caller)
    if (const char* e = std::getenv("DMRG_TILE_SHAPE")) {
      const std::string v(e);
      shape = v == "128x64" ? TILE_128x64 : v == "64x128" ? TILE_64x128 : TILE_64x64;
    }
  }
  F.shape = shape;
  const long TR = tile_rows(shape), TC = tile_cols(shape);
  double total = 0;
  for (size_t j = 0; j < shapes.size(); ++j) {
    const long m = fold == FOLD_M ? long(shapes[j].first) * batch : shapes[j].first;
    const long n = fold == FOLD_N ? long(shapes[j].second) * batch : shapes[j].second;
    tiles_of[j] = ((m + TR - 1) / TR) * ((n + TC - 1) / TC);
    total += double(tiles_of[j]) * double(work_of[j]) * double(entries);
  }
  // about four workgroups per slot of a full chip (256 CUs x 4 resident)
  const double target = std::max(8.0, total / 4096.0);
  std::vector<GTile> tl;
  std::vector<GSeg> sg;
  std::vector<GRed> rd;
  int nslots = 0;
  for (size_t j = 0; j < shapes.size(); ++j) {
    const long m = fold == FOLD_M ? long(shapes[j].first) * batch : shapes[j].first;
    const long n = fold == FOLD_N ? long(shapes[j].second) * batch : shapes[j].second;
    const int tm = int((m + TR - 1) / TR), tn = int((n + TC - 1) / TC);
    const int ncon_j = ranges[j].second - ranges[j].first;
    int nseg = int(std::ceil(double(work_of[j]) / target));
    nseg = std::max(1, std::min(nseg, ncon_j));
    std::vector<std::pair<int, int>> cuts;
    if (nseg > 1) {
      const double per = double(work_of[j]) / nseg;
      int c = ranges[j].first;
      double acc = 0;
      int start = c;
      for (; c < ranges[j].second; ++c) {
        acc += (con_k[c] + 31) / 32;
        if (acc >= per * double(cuts.size() + 1) && int(cuts.size()) < nseg - 1) {
          cuts.push_back({start, c + 1});
          start = c + 1;
        }
      }
      if (start < ranges[j].second) cuts.push_back({start, ranges[j].second});
      nseg = int(cuts.size());
    }
    for (int a = 0; a < tm; ++a)
      for (int c = 0; c < tn; ++c) {
        if (nseg <= 1) {
          tl.push_back({int(j), a, c, -1});
          continue;
        }
        rd.push_back({int(j), a, c, nslots, nseg, 0});
        for (int q = 0; q < nseg; ++q) {
          tl.push_back({int(j), a, c, int(sg.size())});
          sg.push_back({cuts[q].first, cuts[q].second, nslots + q, 0});
        }
        nslots += nseg;
      }
  }
  upload(x, F.tiles, tl);
  upload(x, F.segs, sg);
  upload(x, F.red, rd);
  F.ntiles = int(tl.size());
  F.nred = int(rd.size());
  F.nslots = nslots;
  return F;
}

void LinCombPlan::launch(Ctx& x, const Bases& b, int batch, int prec) const {
  if (ng)
    launch_lincomb_grouped(prec, g.as<LCGroup>(), ng, t.as<LCTarget>(), u.as<LCSource>(), coef.as<double>(),
                           coef32.as<float>(), max_size, b, batch, x.stream);
  if (nd) {
    if (prec == 0) launch_diag_add_f64(d.as<DiagAdd>(), nd, b, batch, x.stream);
    else launch_diag_add_f32(d.as<DiagAdd>(), nd, b, batch, x.stream);
  }
  DMRG_HIP(hipGetLastError());
}

namespace {

struct LinCombBuilder {
  std::vector<LCTarget> t;
  std::vector<LCSource> s;
  std::vector<DiagAdd> d;
  long max_size = 0;
  void target(int base, long off, long size, bool acc) {
    t.push_back({off, size, base, int(s.size()), int(s.size()), acc ? 1 : 0});
    max_size = std::max(max_size, size);
  }
  void source(int base, long off, double c) {
    s.push_back({off, base, 0, c});
    t.back().s1 = int(s.size());
  }
  // Targets of equal size are grouped by similar source lists, kLCGroup at
  // a time; each group reads the merged source list once.
  void finish(Ctx& x, LinCombPlan& P) {
    typedef std::pair<int, long> SrcKey;  // (base, offset)
    std::vector<std::vector<SrcKey>> keys(t.size());
    for (size_t k = 0; k < t.size(); ++k) {
      for (int j = t[k].s0; j < t[k].s1; ++j) keys[k].push_back({s[j].base, s[j].off});
      std::sort(keys[k].begin(), keys[k].end());
    }
    std::map<long, std::vector<int>> by_size;
    for (size_t k = 0; k < t.size(); ++k) by_size[t[k].size].push_back(int(k));
    std::vector<LCTarget> tg;
    std::vector<LCGroup> gr;
    std::vector<LCSource> us;
    std::vector<double> cf;
    for (auto& kv : by_size) {
      std::vector<int>& v = kv.second;
      std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return keys[a] < keys[b]; });
      for (size_t g0 = 0; g0 < v.size(); g0 += kLCGroup) {
        const int n = int(std::min<size_t>(kLCGroup, v.size() - g0));
        std::map<SrcKey, std::vector<double>> uni;
        for (int k = 0; k < n; ++k) {
          const LCTarget& q = t[v[g0 + k]];
          for (int j = q.s0; j < q.s1; ++j) {
            auto& c = uni[{s[j].base, s[j].off}];
            if (c.empty()) c.assign(kLCGroup, 0.0);
            c[k] += s[j].c;
          }
        }
        LCGroup G{kv.first, int(tg.size()), n, int(us.size()), 0, 0};
        for (int k = 0; k < n; ++k) tg.push_back(t[v[g0 + k]]);
        for (auto& u : uni) {
          us.push_back({u.first.second, u.first.first, 0, 0.0});
          cf.insert(cf.end(), u.second.begin(), u.second.end());
        }
        G.u1 = int(us.size());
        gr.push_back(G);
        P.reads += double(kv.first) * double(uni.size());
      }
    }
    upload(x, P.t, tg);
    upload(x, P.u, us);
    upload(x, P.coef, cf);
    upload(x, P.coef32, std::vector<float>(cf.begin(), cf.end()));
    upload(x, P.g, gr);
    upload(x, P.d, d);
    P.nt = int(tg.size());
    P.ng = int(gr.size());
    P.nd = int(d.size());
    P.max_size = max_size;
    for (auto& q : t) P.elems += double(q.size);
  }
};

void make_gemm_plan(Ctx& x, GemmPlan& P, std::vector<GJob>& jobs, std::vector<std::vector<GContrib>>& per,
                    const std::vector<int>& gather = {}) {
  std::vector<GContrib> con;
  std::vector<GTile> tiles;
  double fl = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    jobs[j].c0 = int(con.size());
    for (auto& c : per[j]) {
      con.push_back(c);
      if (!(c.flags & GC_A_IDENTITY)) fl += 2.0 * jobs[j].m * jobs[j].n * c.k;
    }
    jobs[j].c1 = int(con.size());
    const int tm = (jobs[j].m + 63) / 64, tn = (jobs[j].n + 63) / 64;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) tiles.push_back({int(j), a, b, 0});
    P.shapes.push_back({jobs[j].m, jobs[j].n});
    P.elems_c += double(jobs[j].m) * jobs[j].n;
    P.ranges.push_back({jobs[j].c0, jobs[j].c1});
    for (int c = jobs[j].c0; c < jobs[j].c1; ++c) P.con_k.push_back(con[c].k);
    P.mask_c |= 1u << jobs[j].baseC;
    long kc = 0;
    for (int c = jobs[j].c0; c < jobs[j].c1; ++c) kc += (con[c].k + 31) / 32;
    P.ncon += jobs[j].c1 - jobs[j].c0;
    P.kchunks += kc;
    P.kchunks_max = std::max(P.kchunks_max, kc);
    for (int c = jobs[j].c0; c < jobs[j].c1; ++c) {
      if (!(con[c].flags & GC_A_IDENTITY)) P.mask_a |= 1u << con[c].baseA;
      P.mask_b |= 1u << con[c].baseB;
    }
    const int gf = jobs[j].flags & (GJ_GATHER_A | GJ_GATHER_B);
    if (gf) {
      // a gathered operand: one contribution, rows of A contiguous in k
      // (gather A) or columns of B contiguous in k (gather B)
      DMRG_REQUIRE(gf != (GJ_GATHER_A | GJ_GATHER_B) && jobs[j].c1 - jobs[j].c0 == 1, DMRG_ERR_INTERNAL,
                   "gathered job with several contributions");
      const GContrib& c = con[jobs[j].c0];
      const long len = gf == GJ_GATHER_A ? jobs[j].m : jobs[j].n;
      DMRG_REQUIRE(gf == GJ_GATHER_A ? !(c.flags & (GC_TRANS_A | GC_A_IDENTITY)) : (c.flags & GC_TRANS_B) != 0,
                   DMRG_ERR_INTERNAL, "gathered operand not contiguous in k");
      DMRG_REQUIRE(jobs[j].pad >= 0 && long(jobs[j].pad) + len <= long(gather.size()), DMRG_ERR_INTERNAL,
                   "gather entries out of range");
    }
  }
  {
    std::set<std::pair<int, long>> seen_a, seen_b;
    for (size_t j = 0; j < jobs.size(); ++j)
      for (int c = jobs[j].c0; c < jobs[j].c1; ++c) {
        // a gathered operand has its own rows / columns (offset 0 is not a key)
        const bool ga = jobs[j].flags & GJ_GATHER_A, gb = jobs[j].flags & GJ_GATHER_B;
        if (!(con[c].flags & GC_A_IDENTITY) && (ga || seen_a.insert({con[c].baseA, con[c].offA}).second))
          P.elems_a += double(jobs[j].m) * con[c].k;
        if (gb || seen_b.insert({con[c].baseB, con[c].offB}).second) P.elems_b += double(con[c].k) * jobs[j].n;
      }
  }
  upload(x, P.tiles, tiles);
  upload(x, P.jobs, jobs);
  upload(x, P.con, con);
  upload(x, P.gat, gather);
  P.ntiles = int(tiles.size());
  P.flops = fl;
}

// Stage-1 items that share one operand are merged into one job whose other
// operand is gathered: rows stacked (merge 1, the products sit one below the
// other with their own leading dimension) or columns side by side (merge 2,
// the products become column ranges of one matrix whose leading dimension is
// the total width).  A merged job fills its tiles across many small products
// instead of padding each to a tile.  Merged groups are capped at an eighth
// of the workspace budget so that chunks stay well packed.
namespace {
struct T1Group {
  int merge = 0;
  std::vector<int> items;
  long elems = 0, len = 0;  // workspace elements; stacked rows / total columns
};

bool mergeable(const TwoStageBuilder::T1& t) {
  const GContrib& c = t.con;
  if (t.merge == 1) {
    if (c.flags & (GC_TRANS_A | GC_A_IDENTITY)) return false;
    return c.offA >= 0 && c.offA + long(t.job.m - 1) * c.lda + c.k <= 0x7fffffffL;
  }
  if (t.merge == 2) {
    if (!(c.flags & GC_TRANS_B)) return false;
    return c.offB >= 0 && c.offB + long(t.job.n - 1) * c.ldb + c.k <= 0x7fffffffL;
  }
  return false;
}
}  // namespace

// Split the stage-1 items into chunks whose workspace fits the budget and
// build the two device lists of each chunk.
void finish_two_stage(Ctx& x, TwoStageBuilder& B, TwoStagePlan& P, bool overwrite) {
  const long budget = x.t_budget_per_vec;
  const long cap = std::max(1L, budget / 8);
  // group the items: key = the shared operand and everything a merged job
  // has in common (flags, inner length, leading dimensions, the unmerged
  // output dimension, alpha)
  typedef std::tuple<int, int, int, int, long, int, int, int, int, double> GKey;
  std::map<GKey, int> open;
  std::vector<T1Group> groups;
  for (size_t k = 0; k < B.t1.size(); ++k) {
    const TwoStageBuilder::T1& t = B.t1[k];
    const int mg = mergeable(t) ? t.merge : 0;
    int gi = -1;
    GKey key;
    if (mg) {
      const GContrib& c = t.con;
      key = mg == 1 ? GKey(1, c.flags, c.k, c.baseB, c.offB, c.ldb, c.baseA, c.lda, t.job.n, c.alpha)
                    : GKey(2, c.flags, c.k, c.baseA, c.offA, c.lda, c.baseB, c.ldb, t.job.m, c.alpha);
      auto it = open.find(key);
      if (it != open.end() && groups[it->second].elems + t.elems <= cap) gi = it->second;
    }
    if (gi < 0) {
      groups.emplace_back();
      gi = int(groups.size()) - 1;
      groups[gi].merge = mg;
      if (mg) open[key] = gi;
    }
    T1Group& g = groups[gi];
    g.items.push_back(int(k));
    g.elems += t.elems;
    g.len += mg == 1 ? t.job.m : t.job.n;
  }
  std::vector<int> chunk_of(B.t1.size()), gchunk(groups.size());
  std::vector<long> toff(B.t1.size()), ldt(B.t1.size(), 0), goff(groups.size());
  long used = 0;
  int nch = 0;
  for (size_t q = 0; q < groups.size(); ++q) {
    if (q == 0 || (used + groups[q].elems > budget && used > 0)) {
      ++nch;
      used = 0;
    }
    gchunk[q] = nch - 1;
    goff[q] = used;
    long pos = 0;  // row (merge 1) or column (merge 2) of each item in its group
    for (int k : groups[q].items) {
      const TwoStageBuilder::T1& t = B.t1[k];
      chunk_of[k] = nch - 1;
      if (groups[q].merge == 2) {
        toff[k] = used + pos;
        ldt[k] = groups[q].len;
        pos += t.job.n;
      } else {
        toff[k] = used + pos * t.job.ldc;
        pos += t.job.m;
      }
    }
    used += groups[q].elems;
    P.t_per_vec = std::max(P.t_per_vec, used);
  }
  if (nch == 0) nch = 1;
  P.chunks.clear();
  P.chunks.resize(nch);
  P.flops1 = P.flops2 = 0;
  for (int c = 0; c < nch; ++c) {
    std::vector<GJob> j1;
    std::vector<std::vector<GContrib>> p1;
    std::vector<int> gat;
    for (size_t q = 0; q < groups.size(); ++q) {
      if (gchunk[q] != c) continue;
      const T1Group& g = groups[q];
      if (g.merge == 0 || g.items.size() == 1) {
        for (int k : g.items) {
          GJob j = B.t1[k].job;
          j.offC = toff[k];
          j.baseC = B_T;
          j.flags = 0;
          j1.push_back(j);
          p1.push_back({B.t1[k].con});
        }
        continue;
      }
      const TwoStageBuilder::T1& f = B.t1[g.items.front()];
      GJob j = f.job;
      GContrib con = f.con;
      j.offC = goff[q];
      j.baseC = B_T;
      j.pad = int(gat.size());
      if (g.merge == 1) {
        j.m = int(g.len);
        j.flags = GJ_GATHER_A;
        con.offA = 0;
        for (int k : g.items) {
          const TwoStageBuilder::T1& t = B.t1[k];
          for (int r = 0; r < t.job.m; ++r) gat.push_back(int(t.con.offA + long(r) * t.con.lda));
        }
      } else {
        j.n = int(g.len);
        j.ldc = int(g.len);
        j.flags = GJ_GATHER_B;
        con.offB = 0;
        for (int k : g.items) {
          const TwoStageBuilder::T1& t = B.t1[k];
          for (int r = 0; r < t.job.n; ++r) gat.push_back(int(t.con.offB + long(r) * t.con.ldb));
        }
      }
      j1.push_back(j);
      p1.push_back({con});
    }
    make_gemm_plan(x, P.chunks[c].first, j1, p1, gat);
    std::vector<GJob> j2;
    std::vector<std::vector<GContrib>> p2;
    std::map<std::pair<int, long>, int> job_of;
    auto job = [&](int base, long off, int ldc, int m, int n) {
      auto key = std::make_pair(base, off);
      auto it = job_of.find(key);
      if (it != job_of.end()) return it->second;
      GJob g{};
      g.offC = off;
      g.baseC = base;
      g.ldc = ldc;
      g.m = m;
      g.n = n;
      g.flags = (overwrite && c == 0) ? 0 : GJ_ACCUMULATE;
      j2.push_back(g);
      p2.emplace_back();
      job_of[key] = int(j2.size()) - 1;
      return int(j2.size()) - 1;
    };
    if (overwrite && c == 0)
      for (auto& o : B.outputs) job(std::get<1>(o), std::get<0>(o), std::get<2>(o), std::get<3>(o), std::get<4>(o));
    for (auto& s : B.s2) {
      const int ck = s.t1 >= 0 ? chunk_of[s.t1] : 0;
      if (ck != c) continue;
      GContrib g = s.con;
      if (s.t1 >= 0 && s.t_is_a) {
        g.offA += toff[s.t1];
        g.baseA = B_T;
        if (ldt[s.t1]) g.lda = int(ldt[s.t1]);
      } else if (s.t1 >= 0) {
        g.offB += toff[s.t1];
        g.baseB = B_T;
        if (ldt[s.t1]) g.ldb = int(ldt[s.t1]);
      }
      p2[job(s.baseC, s.offC, s.ldc, s.m, s.n)].push_back(g);
    }
    make_gemm_plan(x, P.chunks[c].second, j2, p2);
    P.flops1 += P.chunks[c].first.flops;
    P.flops2 += P.chunks[c].second.flops;
  }
}

}  // namespace

void log_jsonl(const std::string& json_object) {
  const char* path = std::getenv("DMRG_LOG_JSONL");
  if (!path || !*path) return;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (FILE* f = std::fopen(path, "a")) {
    std::fputs(json_object.c_str(), f);
    std::fputc('\n', f);
    std::fclose(f);
  }
}

void build_gemm_plan(Ctx& x, GemmPlan& P, std::vector<GJob>& jobs, std::vector<std::vector<GContrib>>& per,
                     const std::vector<int>& gather) {
  make_gemm_plan(x, P, jobs, per, gather);
}

void print_plan_stats(const char* what, int i, int width, const ContractionPlan& P) {
  long jobs1 = 0, con1 = 0, kc1 = 0, jobs2 = 0, con2 = 0, kc2 = 0, kmax2 = 0;
  for (auto& ch : P.main.chunks) {
    jobs1 += long(ch.first.shapes.size());
    con1 += ch.first.ncon;
    kc1 += ch.first.kchunks;
    jobs2 += long(ch.second.shapes.size());
    con2 += ch.second.ncon;
    kc2 += ch.second.kchunks;
    kmax2 = std::max(kmax2, ch.second.kchunks_max);
  }
  // stage-2 traffic model for 16 vectors folded into N (64x64 tiles, K
  // padded to chunks of 16): operand elements streamed by the tiles, the
  // distinct operand elements, and executed / algorithmic MFMA work
  {
    const int nb = 16;
    double tile_reads = 0, distinct = 0, exec = 0, algo = 0;
    for (auto& ch : P.main.chunks) {
      const GemmPlan& G = ch.second;
      distinct += G.elems_a + G.elems_b * nb;
      for (size_t j = 0; j < G.shapes.size(); ++j) {
        const long m = G.shapes[j].first, n = long(G.shapes[j].second) * nb;
        const long tiles = ((m + 63) / 64) * ((n + 63) / 64);
        long kp = 0, k = 0;
        for (int c = G.ranges[j].first; c < G.ranges[j].second; ++c) {
          kp += (G.con_k[c] + 15) / 16 * 16;
          k += G.con_k[c];
        }
        tile_reads += double(tiles) * 128.0 * double(kp);
        exec += double(tiles) * 2.0 * 64 * 64 * double(kp);
        algo += 2.0 * double(m) * double(n) * double(k);
      }
    }
    std::fprintf(stderr, "[plan] %s site %d stage-2 model (16 vectors, N fold): tile operand reads %.3g elems, "
                 "distinct %.3g (x%.1f), executed/algorithmic MFMA %.2f\n", what, i, tile_reads, distinct,
                 tile_reads / std::max(distinct, 1.0), exec / std::max(algo, 1.0));
  }
  std::fprintf(stderr,
               "[plan] %s site %d width %d: form targets %d elems %.3g reads %.3g | chunks %zu | stage1 jobs %ld "
               "contribs %ld kchunks %ld flops %.3g | stage2 jobs %ld contribs %ld kchunks %ld max/job %ld flops %.3g | "
               "post targets %d reads %.3g\n",
               what, i, width, P.form.nt, P.form.elems, P.form.reads, P.main.chunks.size(), jobs1, con1, kc1,
               P.main.flops1,
               jobs2, con2, kc2, kmax2, P.main.flops2, P.post.nt, P.post.reads);
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
  const char* env = std::getenv("DMRG_T_BUDGET_PER_VEC");
  t_budget_per_vec = env ? std::max(1L, std::atol(env)) : (32L << 20);
  // FP64 contractions: matrix cores (default) or the plain FMA kernel
  const char* g = std::getenv("DMRG_FP64_GEMM");
  fp64_mfma = !(g && std::string(g) == "fma");
  for (auto& a : tile_policy)
    for (auto& b : a)
      for (int& c : b) c = -1;
  if (device >= 0) {
    DMRG_HIP(hipSetDevice(device));
    scratch_ = scratch_address(device);
  }
  H.reset(new QCHamiltonian(L, h, eri, ecore));
}

Ctx::~Ctx() {
  for (hipEvent_t e : main_events_) (void)hipEventDestroy(e);
  for (auto& f : fo_chain) f.reset();
  drop_gauge_kit();
  clear_plans();
  left.clear();
  right.clear();
  site.clear();
}

void Ctx::clear_plans() {
  renorm_plans_.clear();
  sigma_plans_.clear();
  diag_plans_.clear();
}

void Ctx::require_gpu() const {
  DMRG_REQUIRE(device >= 0, DMRG_ERR_STATE, "host-only context: no device calls");
}

void Ctx::sync() { DMRG_HIP(hipStreamSynchronize(stream)); }

void* Ctx::dev_alloc(size_t bytes) {
  require_gpu();
  DMRG_REQUIRE(!no_alloc_, DMRG_ERR_STATE,
               "dmrg_sigma_noalloc would allocate device memory (plans, tile lists or FP32 operator copies are "
               "missing): call dmrg_sigma once with the same site, kind, nvec and precision first");
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
  {
    std::lock_guard<std::mutex> lock(op_layout_mu_);
    auto it = op_layouts_.find(key);
    if (it != op_layouts_.end()) return it->second.get();
  }
  // built outside the lock; a concurrent builder of the same key keeps the
  // first entry
  auto O = std::make_unique<OpLayout>();
  build_op_layout(*O, bonds[bond], dna, dnb);
  std::lock_guard<std::mutex> lock(op_layout_mu_);
  auto& slot = op_layouts_[key];
  if (!slot) slot = std::move(O);
  return slot.get();
}

long Ctx::bond_offset(int b, int sector) const {
  long o = 0;
  for (int s = 0; s < sector; ++s) o += bonds[b].dim[s];
  return o;
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
  clear_plans();
  drop_gauge_kit();
  for (auto& f : fo_chain) f.reset();
  ++generation;
  bonds = std::move(B);
  layouts_.clear();
  op_layouts_.clear();
  left.clear();
  right.clear();
  ops_prec = -1;
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
  upload_lambda();
}

void Ctx::upload_lambda() {
  lam_dev.clear();
  laminv_dev.clear();
  lam_dev.resize(L + 1);
  laminv_dev.resize(L + 1);
  for (int b = 0; b <= L; ++b) upload_lambda_bond(b);
}

void Ctx::upload_lambda_bond(int b) {
  std::vector<double> v, vi;
  double mx = 0;
  for (auto& s : lam[b])
    for (double x : s) mx = std::max(mx, std::fabs(x));
  for (auto& s : lam[b])
    for (double x : s) {
      v.push_back(x);
      vi.push_back(std::fabs(x) > 1e-14 * mx ? 1.0 / x : 0.0);
    }
  upload(*this, lam_dev[b], v);
  upload(*this, laminv_dev[b], vi);
}

void Ctx::invalidate_bond(int b) {
  auto touches = [b](int i, int w) { return b == i || b == i + w; };
  for (auto it = sigma_plans_.begin(); it != sigma_plans_.end();)
    it = touches(std::get<0>(it->first), std::get<1>(it->first)) ? sigma_plans_.erase(it) : std::next(it);
  for (auto it = diag_plans_.begin(); it != diag_plans_.end();)
    it = touches(it->first.first, it->first.second) ? diag_plans_.erase(it) : std::next(it);
  for (auto it = renorm_plans_.begin(); it != renorm_plans_.end();)
    it = touches(std::get<1>(it->first), 1) ? renorm_plans_.erase(it) : std::next(it);
  for (auto it = layouts_.begin(); it != layouts_.end();)
    it = touches(it->first.first, it->first.second) ? layouts_.erase(it) : std::next(it);
  if (b < int(left.size())) left[b] = OpSet();
  if (b < int(right.size())) right[b] = OpSet();
  for (auto it = op_layouts_.begin(); it != op_layouts_.end();)
    it = std::get<0>(it->first) == b ? op_layouts_.erase(it) : std::next(it);
}

void Ctx::set_bond(int b, Bond nb, std::vector<std::vector<double>> lam_b) {
  ++generation;
  invalidate_bond(b);
  drop_gauge_kit();
  for (auto& f : fo_chain) f.reset();
  bonds[b] = std::move(nb);
  lam[b] = std::move(lam_b);
  if (int(lam_dev.size()) == L + 1) upload_lambda_bond(b);
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

long Ctx::opset_size(int bond, int side) {
  const BondChannels& B = side == 0 ? H->left_channels(bond) : H->right_channels(bond);
  const uint64_t ident = side == 0 ? chan_key(CH_ID_H, -1, -1) : chan_key(CH_H_ID, -1, -1);
  long n = 0;
  for (size_t w = 0; w < B.ch.size(); ++w)
    if (B.ch[w].key != ident) n += long(op_layout(bond, B.ch[w].dna, B.ch[w].dnb)->size);
  return n;
}

void Ctx::alloc_opset(OpSet& S, int bond, int side, int nvec, bool first_order, bool reuse, bool f32) {
  const BondChannels& B = side == 0 ? H->left_channels(bond) : H->right_channels(bond);
  S.bond = bond;
  S.side = side;
  S.nvec = nvec;
  S.f32_valid = false;
  S.f32 = f32;
  S.first_order = first_order;
  const uint64_t ident = side == 0 ? chan_key(CH_ID_H, -1, -1) : chan_key(CH_H_ID, -1, -1);
  S.kind.assign(B.ch.size(), REF_OP);
  S.off.assign(B.ch.size(), 0);
  S.lay.assign(B.ch.size(), nullptr);
  long off = 0;
  std::map<std::pair<int, int>, std::vector<int>> by_shift;  // classes contiguous
  for (size_t w = 0; w < B.ch.size(); ++w) {
    if (B.ch[w].key == ident) {
      S.kind[w] = first_order ? REF_ZERO : REF_IDENTITY;
      continue;
    }
    by_shift[{B.ch[w].dna, B.ch[w].dnb}].push_back(int(w));
  }
  for (auto& kv : by_shift) {
    const OpLayout* lay = op_layout(bond, kv.first.first, kv.first.second);
    for (int w : kv.second) {
      S.lay[w] = lay;
      S.off[w] = off;
      off += long(lay->size);
    }
  }
  S.per_vec = off;
  const size_t bytes = std::max<size_t>(size_t(off) * nvec, 1) * (f32 ? 4 : 8);
  if (!reuse || S.data.bytes < bytes) S.data.alloc(this, bytes);
}

// ---------------------------------------------------------------- planning helpers

namespace {

struct Group {
  int key_ch;
  int sid;
  std::vector<std::pair<int, double>> src;
};

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

inline bool has_blk(const ORef& r, int ket) { return r.kind == REF_IDENTITY || r.lay->by_ket[ket] >= 0; }
inline int opbra(const ORef& r, int ket) {
  if (r.kind == REF_IDENTITY) return ket;
  const int b = r.lay->by_ket[ket];
  return b < 0 ? -1 : r.lay->blk[b].bra;
}
inline long opoff(const ORef& r, int ket) { return r.off + long(r.lay->blk[r.lay->by_ket[ket]].off); }

using Sources = std::vector<std::pair<ORef, double>>;

// pool of dressed operators / building blocks inside one base
struct Pool {
  int base;
  long size = 0;
  ORef add(const OpLayout* lay) {
    ORef r;
    r.kind = REF_OP;
    r.base = base;
    r.off = size;
    r.lay = lay;
    size += long(lay->size);
    return r;
  }
};

void emit_formation(LinCombBuilder& lc, const ORef& out, const Sources& srcs) {
  lc.target(out.base, out.off, long(out.lay->size), false);
  double cid = 0.0;
  for (auto& s : srcs) {
    if (s.first.kind == REF_IDENTITY) cid += s.second;
    else if (s.first.kind == REF_OP) lc.source(s.first.base, s.first.off, s.second);
  }
  if (cid != 0.0) {
    DMRG_REQUIRE(out.lay->dna == 0 && out.lay->dnb == 0, DMRG_ERR_INTERNAL, "identity in a shifted class");
    for (auto& b : out.lay->blk)
      if (b.ket == b.bra) lc.d.push_back({out.off + long(b.off), out.base, b.rows, cid, 0});
  }
}

struct RJob {
  ORef X;
  double alpha;
  int sid;
  ORef tgt;
  int pz;
};

}  // namespace

// Renormalization plan.  Per target group the sources are combined either
// before the one-site transform (one dressed operator per target) or after it
// (one transformed building block per shared source, then a linear
// combination), whichever needs fewer transforms.
// bra_first: the kets are batched and the sources and the bra are shared, so
// stage 1 forms U = A_bra^T X (left) or R_bra Z (right) once for all kets and
// stage 2 multiplies U by each ket; otherwise stage 1 forms T = X A_ket
// (left) or Z R_ket^T (right) per ket and stage 2 applies the bra.
ContractionPlan& Ctx::renorm_plan(int dir, int i, const OpSet& src, const OpSet& dst, bool bra_first) {
  auto key = std::make_tuple(dir, i, src.first_order ? 1 : 0, bra_first ? 1 : 0);
  auto it = renorm_plans_.find(key);
  if (it != renorm_plans_.end()) return *it->second;
  return *(renorm_plans_[key] = make_renorm_plan(dir, i, src, dst, bra_first));
}

// Builds a renormalization plan without touching the plan cache, so that
// several can be built at once (build_ops): it reads the channel tables, the
// site layout and site operator of site i (prepared beforehand), and the
// operator-layout cache (guarded by its mutex); its device lists are
// uploaded through the allocator, which is safe from several threads.
std::unique_ptr<ContractionPlan> Ctx::make_renorm_plan(int dir, int i, const OpSet& src, const OpSet& dst,
                                                       bool bra_first) {
  auto P = std::make_unique<ContractionPlan>();
  P->bra_first = bra_first;
  const bool leftdir = dir == DMRG_DIR_LEFT;
  const SiteOp& W = leftdir ? H->site_op(i, 1, H->mode_left(i), H->mode_left(i + 1))
                            : H->site_op(i, 1, H->mode_right(i), H->mode_right(i + 1));
  const SiteLayout& S = layout(i, 1);
  const Bond& bl = bonds[i];
  const Bond& br = bonds[i + 1];
  const int tb = leftdir ? i + 1 : i;  // bond of the targets
  const int db = leftdir ? i : i + 1;  // bond of sources / dressed operators
  const BondChannels& Bt = leftdir ? H->left_channels(tb) : H->right_channels(tb);
  const BondChannels& Bs = leftdir ? H->left_channels(db) : H->right_channels(db);
  const int skip = leftdir ? Bt.find(chan_key(CH_ID_H, -1, -1)) : Bt.find(chan_key(CH_H_ID, -1, -1));
  std::vector<Group> G = group_entries(W, leftdir, skip);
  for (auto& g : G) {
    std::vector<std::pair<int, double>> keep;
    for (auto& s : g.src)
      if (src.kind[s.first] != REF_ZERO) keep.push_back(s);
    g.src.swap(keep);
  }
  std::map<std::pair<int, int>, int> fan;
  for (auto& g : G)
    for (auto& s : g.src) fan[{s.first, g.sid}]++;
  Pool dressed{B_DRESS}, blocks{B_BLK};
  std::vector<std::pair<ORef, Sources>> pend;
  std::vector<RJob> jobs;
  std::map<std::pair<int, int>, ORef> block_of;
  std::vector<std::tuple<ORef, ORef, double>> combine;  // target, block, c
  for (auto& g : G) {
    if (g.src.empty()) continue;
    double share = 0;
    for (auto& s : g.src) share += 1.0 / fan[{s.first, g.sid}];
    const bool after = g.src.size() > 1 && share < 1.0 - 1e-9;
    const DotString& ds = H->dot_string(1, g.sid);
    const ORef tgt = dst.ref(g.key_ch, B_DST);
    const Channel& tch = Bt.ch[g.key_ch];
    if (!after) {
      const int pz = leftdir ? 0 : Bs.ch[g.src[0].first].parity;
      if (g.src.size() == 1) {
        jobs.push_back({src.ref(g.src[0].first, B_SRC), g.src[0].second, g.sid, tgt, pz});
      } else {
        Sources ss;
        for (auto& s : g.src) ss.push_back({src.ref(s.first, B_SRC), s.second});
        const int sa = leftdir ? tch.dna - ds.dna : tch.dna + ds.dna;
        const int sb = leftdir ? tch.dnb - ds.dnb : tch.dnb + ds.dnb;
        ORef d = dressed.add(op_layout(db, sa, sb));
        pend.push_back({d, std::move(ss)});
        jobs.push_back({d, 1.0, g.sid, tgt, pz});
      }
    } else {
      for (auto& s : g.src) {
        auto k2 = std::make_pair(s.first, g.sid);
        auto f = block_of.find(k2);
        ORef blk;
        if (f == block_of.end()) {
          blk = blocks.add(tgt.lay);
          block_of[k2] = blk;
          jobs.push_back({src.ref(s.first, B_SRC), 1.0, g.sid, blk, leftdir ? 0 : Bs.ch[s.first].parity});
        } else {
          blk = f->second;
        }
        combine.push_back({tgt, blk, s.second});
      }
    }
  }
  LinCombBuilder form;
  for (auto& p : pend) emit_formation(form, p.first, p.second);
  form.finish(*this, P->form);
  P->dressed_per_vec = dressed.size;
  P->blocks_per_vec = blocks.size;
  TwoStageBuilder TB;
  for (auto& j : jobs) {
    const DotString& ds = H->dot_string(1, j.sid);
    for (size_t e = 0; e < ds.val.size(); ++e) {
      const int n = ds.ket[e], np = ds.bra[e];
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, n);
        if (b < 0) continue;
        const int c = S.blk[b].c;
        if (leftdir) {
          // T = X(a'<-a) A_ket(a,n,c);  tgt(c'<-c) += al A_bra(a',n',c')^T T
          if (!has_blk(j.X, a)) continue;
          const int ap = opbra(j.X, a);
          const int bp = S.find(ap, np);
          if (bp < 0) continue;
          const int cp = S.blk[bp].c;
          const int tbk = j.tgt.lay->by_ket[c];
          DMRG_REQUIRE(tbk >= 0 && j.tgt.lay->blk[tbk].bra == cp, DMRG_ERR_INTERNAL, "left renorm block mismatch");
          const double sign = (ds.parity && (bl.q[a].n() & 1)) ? -1.0 : 1.0;
          TwoStageBuilder::S2 s2{};
          s2.offC = j.tgt.off + long(j.tgt.lay->blk[tbk].off);
          s2.baseC = j.tgt.base;
          s2.ldc = S.blk[b].cols;
          s2.m = S.blk[bp].cols;
          s2.n = S.blk[b].cols;
          s2.con = {long(S.blk[bp].off), 0, S.blk[bp].cols, S.blk[b].cols, bl.dim[ap], GC_TRANS_A, B_ABRA, B_AKET,
                    j.alpha * ds.val[e] * sign};
          if (j.X.kind == REF_IDENTITY) {
            s2.t1 = -1;
            s2.con.offB = long(S.blk[b].off);
          } else if (bra_first) {
            // U = A_bra(a',n',c')^T X(a'<-a) (m_c' x m_a);  tgt(c'<-c) += al U A_ket(a,n,c)
            auto tk = std::make_tuple(j.X.base, j.X.off, bp);
            auto f = TB.t1_of.find(tk);
            if (f == TB.t1_of.end()) {
              TwoStageBuilder::T1 t{};
              t.merge = 0;
              t.elems = long(S.blk[bp].cols) * bl.dim[a];
              t.job.ldc = bl.dim[a];
              t.job.m = S.blk[bp].cols;
              t.job.n = bl.dim[a];
              t.con = {long(S.blk[bp].off), opoff(j.X, a), S.blk[bp].cols, bl.dim[a], bl.dim[ap], GC_TRANS_A, B_ABRA,
                       j.X.base, 1.0};
              TB.t1.push_back(t);
              f = TB.t1_of.emplace(tk, int(TB.t1.size()) - 1).first;
            }
            s2.t1 = f->second;
            s2.t_is_a = true;
            s2.con = {0, long(S.blk[b].off), bl.dim[a], S.blk[b].cols, bl.dim[a], 0, B_T, B_AKET,
                      j.alpha * ds.val[e] * sign};
          } else {
            auto tk = std::make_tuple(j.X.base, j.X.off, b);
            auto f = TB.t1_of.find(tk);
            if (f == TB.t1_of.end()) {
              TwoStageBuilder::T1 t{};
              t.merge = 1;  // X blocks share A_ket: stack their rows
              t.elems = long(bl.dim[ap]) * S.blk[b].cols;
              t.job.ldc = S.blk[b].cols;
              t.job.m = bl.dim[ap];
              t.job.n = S.blk[b].cols;
              t.con = {opoff(j.X, a), long(S.blk[b].off), S.blk[b].rows, S.blk[b].cols, S.blk[b].rows, 0, j.X.base,
                       B_AKET, 1.0};
              TB.t1.push_back(t);
              f = TB.t1_of.emplace(tk, int(TB.t1.size()) - 1).first;
            }
            s2.t1 = f->second;
            s2.con.offB = 0;
          }
          TB.s2.push_back(s2);
        } else {
          // T = Z(c'<-c) R_ket(a,n,c)^T;  tgt(a'<-a) += al R_bra(a',n',c') T
          if (!has_blk(j.X, c)) continue;
          const int cp = opbra(j.X, c);
          const QN qnp = site_qn(np);
          const int ap = bl.find(QN{br.q[cp].na - qnp.na, br.q[cp].nb - qnp.nb});
          if (ap < 0) continue;
          const int bp = S.find(ap, np);
          if (bp < 0 || S.blk[bp].c != cp) continue;
          const int tbk = j.tgt.lay->by_ket[a];
          DMRG_REQUIRE(tbk >= 0 && j.tgt.lay->blk[tbk].bra == ap, DMRG_ERR_INTERNAL, "right renorm block mismatch");
          const double sign = (j.pz && (site_qn(n).n() & 1)) ? -1.0 : 1.0;
          TwoStageBuilder::S2 s2{};
          s2.offC = j.tgt.off + long(j.tgt.lay->blk[tbk].off);
          s2.baseC = j.tgt.base;
          s2.ldc = S.blk[b].rows;
          s2.m = S.blk[bp].rows;
          s2.n = S.blk[b].rows;
          if (j.X.kind == REF_IDENTITY) {
            s2.t1 = -1;
            s2.con = {long(S.blk[bp].off), long(S.blk[b].off), S.blk[bp].cols, S.blk[b].cols, S.blk[b].cols,
                      GC_TRANS_B, B_ABRA, B_AKET, j.alpha * ds.val[e] * sign};
          } else if (bra_first) {
            // U = R_bra(a',n',c') Z(c'<-c) (m_a' x m_c);  tgt(a'<-a) += al U R_ket(a,n,c)^T
            auto tk = std::make_tuple(j.X.base, j.X.off, bp);
            auto f = TB.t1_of.find(tk);
            if (f == TB.t1_of.end()) {
              TwoStageBuilder::T1 t{};
              t.merge = 1;  // bra blocks share Z: stack their rows
              t.elems = long(S.blk[bp].rows) * S.blk[b].cols;
              t.job.ldc = S.blk[b].cols;
              t.job.m = S.blk[bp].rows;
              t.job.n = S.blk[b].cols;
              t.con = {long(S.blk[bp].off), opoff(j.X, c), S.blk[bp].cols, S.blk[b].cols, br.dim[cp], 0, B_ABRA,
                       j.X.base, 1.0};
              TB.t1.push_back(t);
              f = TB.t1_of.emplace(tk, int(TB.t1.size()) - 1).first;
            }
            s2.t1 = f->second;
            s2.t_is_a = true;
            s2.con = {0, long(S.blk[b].off), S.blk[b].cols, S.blk[b].cols, S.blk[b].cols, GC_TRANS_B, B_T, B_AKET,
                      j.alpha * ds.val[e] * sign};
          } else {
            auto tk = std::make_tuple(j.X.base, j.X.off, b);
            auto f = TB.t1_of.find(tk);
            if (f == TB.t1_of.end()) {
              TwoStageBuilder::T1 t{};
              t.merge = 1;  // Z blocks share R_ket: stack their rows
              t.elems = long(br.dim[cp]) * S.blk[b].rows;
              t.job.ldc = S.blk[b].rows;
              t.job.m = br.dim[cp];
              t.job.n = S.blk[b].rows;
              t.con = {opoff(j.X, c), long(S.blk[b].off), S.blk[b].cols, S.blk[b].cols, S.blk[b].cols, GC_TRANS_B,
                       j.X.base, B_AKET, 1.0};
              TB.t1.push_back(t);
              f = TB.t1_of.emplace(tk, int(TB.t1.size()) - 1).first;
            }
            s2.t1 = f->second;
            s2.con = {long(S.blk[bp].off), 0, S.blk[bp].cols, S.blk[b].rows, br.dim[cp], 0, B_ABRA, B_T,
                      j.alpha * ds.val[e] * sign};
          }
          TB.s2.push_back(s2);
        }
      }
    }
  }
  finish_two_stage(*this, TB, P->main, false);
  LinCombBuilder post;
  std::map<std::pair<int, long>, std::vector<std::pair<ORef, double>>> by_tgt;
  for (auto& cb : combine)
    by_tgt[{std::get<0>(cb).base, std::get<0>(cb).off}].push_back({std::get<1>(cb), std::get<2>(cb)});
  for (auto& kv : by_tgt) {
    const ORef& first = kv.second.front().first;
    post.target(kv.first.first, kv.first.second, long(first.lay->size), true);
    for (auto& s : kv.second) post.source(s.first.base, s.first.off, s.second);
  }
  post.finish(*this, P->post);
  if (std::getenv("DMRG_PLAN_STATS")) print_plan_stats(dir == 0 ? "renorm-L" : "renorm-R", i, 1, *P);
  return P;
}

void Ctx::renorm(int dir, int i, const double* Abra, const double* Aket, long aket_stride, const OpSet& src,
                 OpSet& dst, bool accumulate, int batch, int prec, long abra_stride) {
  const bool src_b = src.nvec > 1, ket_b = aket_stride != 0, bra_b = abra_stride != 0;
  DMRG_REQUIRE(!bra_b || (!ket_b && !src_b), DMRG_ERR_INTERNAL, "batched bra with a batched ket or source");
  // a batched bra takes the plan that forms T = X A_ket (shared here) in
  // stage 1 and applies the bra in stage 2, where each entry reads its own
  ContractionPlan& P = renorm_plan(dir, i, src, dst, ket_b && !src_b && batch > 1);
  // stage-1 products: per ket unless formed from the bra (shared); the
  // results (and the building blocks) are per entry whenever a source, the
  // ket or the bra is
  const bool t_b = P.bra_first ? src_b : (src_b || ket_b);
  const bool o_b = src_b || ket_b || bra_b;
  const size_t esz = prec == DMRG_FP64 ? 8 : 4;
  Bases b{};
  b.p[B_ABRA] = const_cast<double*>(Abra);
  b.stride[B_ABRA] = abra_stride;
  b.p[B_AKET] = const_cast<double*>(Aket);
  b.stride[B_AKET] = aket_stride;
  b.p[B_SRC] = src.ptr();
  b.stride[B_SRC] = src_b ? src.per_vec : 0;
  b.p[B_DST] = dst.ptr();
  b.stride[B_DST] = dst.nvec > 1 ? dst.per_vec : 0;
  ws_dress.ensure(this, std::max<size_t>(size_t(P.dressed_per_vec) * (src_b ? batch : 1), 1) * esz);
  // an FP32 destination takes FP32 building blocks and an FP32 combination
  const bool dst32 = dst.f32;
  DMRG_REQUIRE(prec != DMRG_FP64 || (!src.f32 && !dst32), DMRG_ERR_INTERNAL, "FP32 operator set in an FP64 renormalization");
  ws_blk.ensure(this, std::max<size_t>(size_t(P.blocks_per_vec) * (o_b ? batch : 1), 1) * (dst32 ? 4 : 8));
  ws_T.ensure(this, std::max<size_t>(size_t(P.main.t_per_vec) * (t_b ? batch : 1), 1) * esz);
  b.p[B_DRESS] = ws_dress.as<double>();
  b.stride[B_DRESS] = src_b ? P.dressed_per_vec : 0;
  b.p[B_BLK] = ws_blk.as<double>();
  b.stride[B_BLK] = o_b ? P.blocks_per_vec : 0;
  b.p[B_T] = ws_T.as<double>();
  b.stride[B_T] = t_b ? P.main.t_per_vec : 0;
  if (prec != DMRG_FP64) {
    // FP32 operands: operator shadow, site tensors converted per call
    b.p[B_SRC] = reinterpret_cast<double*>(f32_data(src));
    const long S = long(layout(i, 1).size);
    const long nket = ket_b ? S * batch : S;
    const long nbra = bra_b ? S * batch : S;
    DMRG_REQUIRE((!ket_b || aket_stride == S) && (!bra_b || abra_stride == S), DMRG_ERR_INTERNAL,
                 "batched site tensors must be contiguous in FP32 renormalization");
    ws_a32.ensure(this, size_t(nbra + nket) * 4);
    float* abra = ws_a32.as<float>();
    float* aket = abra + nbra;
    launch_convert_f64_f32(Abra, abra, nbra, stream);
    launch_convert_f64_f32(Aket, aket, nket, stream);
    b.p[B_ABRA] = reinterpret_cast<double*>(abra);
    b.p[B_AKET] = reinterpret_cast<double*>(aket);
    b.stride[B_ABRA] = bra_b ? S : 0;
    b.stride[B_AKET] = ket_b ? S : 0;
  }
  dst.f32_valid = false;
  const long nblk = P.blocks_per_vec * (o_b ? batch : 1);
  if (dst32) {
    if (!accumulate) launch_fill_f32(dst.data.as<float>(), long(dst.per_vec) * dst.nvec, stream);
    if (nblk) launch_fill_f32(ws_blk.as<float>(), nblk, stream);
  } else {
    if (!accumulate) launch_fill_f64(dst.ptr(), long(dst.per_vec) * dst.nvec, 0.0, stream);
    if (nblk) launch_fill_f64(ws_blk.as<double>(), nblk, 0.0, stream);
  }
  P.form.launch(*this, b, src_b ? batch : 1, prec);
  // both stages run with the products tag: the block-cyclic XCD order of
  // that instantiation is faster for the renormalization's accumulation
  for (auto& ch : P.main.chunks) {
    ch.first.launch(*this, b, t_b ? batch : 1, prec, prec == DMRG_FP64);
    ch.second.launch(*this, b, batch, prec, !dst32);
  }
  P.post.launch(*this, b, batch, dst32 ? DMRG_FP32 : DMRG_FP64);
  stats.renorm_flops += P.main.flops1 * (t_b ? batch : 1) + P.main.flops2 * batch;
}

void Ctx::build_ops(int prec) {
  require_gpu();
  DMRG_REQUIRE(have_mps, DMRG_ERR_STATE, "import or compute an MPS first");
  DMRG_REQUIRE(prec == DMRG_FP64 || prec == DMRG_FP32 || prec == DMRG_BF16X3, DMRG_ERR_INVALID_ARG,
               "unsupported precision");
  // The zeroth-order pools feed every later contraction and their errors
  // compound over the bonds, so a BF16x3 request builds them in FP32; the
  // sigma and the first-order sets of the TDA use BF16x3 as asked.
  const int rprec = prec == DMRG_BF16X3 ? DMRG_FP32 : prec;
  left.clear();
  right.clear();
  left.resize(L + 1);
  right.resize(L + 1);
  for (auto& f : fo_chain) f.reset();
  ++generation;
  stats.renorm_flops = 0;
  // all sets and plans first (host planning, timed apart), then the
  // renormalizations back to back on the stream
  const auto h0 = std::chrono::steady_clock::now();
  parallel_for(2 * (L + 1), [&](int t) {
    const int b = t / 2;
    if (t % 2 == 0) alloc_opset(left[b], b, 0, 1, false);
    else alloc_opset(right[b], b, 1, 1, false);
  });
  // the 2L plans are independent: built on a pool of host threads after the
  // shared lazily built objects they read (site layouts and site
  // operators) exist, then entered into the cache
  for (int i = 0; i < L; ++i) layout(i, 1);
  parallel_for(2 * L, [&](int t) {
    const int i = t / 2;
    if (t % 2 == 0) H->site_op(i, 1, H->mode_left(i), H->mode_left(i + 1));
    else H->site_op(i, 1, H->mode_right(i), H->mode_right(i + 1));
  });
  {
    std::vector<std::function<std::unique_ptr<ContractionPlan>()>> fns;
    for (int i = 0; i < L; ++i)
      fns.push_back([this, i]() { return make_renorm_plan(DMRG_DIR_LEFT, i, left[i], left[i + 1], false); });
    for (int i = L - 1; i >= 0; --i)
      fns.push_back([this, i]() { return make_renorm_plan(DMRG_DIR_RIGHT, i, right[i + 1], right[i], false); });
    auto built = build_parallel(fns);
    for (int t = 0; t < 2 * L; ++t) {
      const int i = t < L ? t : 2 * L - 1 - t;
      renorm_plans_[std::make_tuple(t < L ? DMRG_DIR_LEFT : DMRG_DIR_RIGHT, i, 0, 0)] = std::move(built[t]);
    }
  }
  stats.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
  hipEvent_t e0, e1;
  DMRG_HIP(hipEventCreate(&e0));
  DMRG_HIP(hipEventCreate(&e1));
  DMRG_HIP(hipEventRecord(e0, stream));
  for (int i = 0; i < L; ++i)
    renorm(DMRG_DIR_LEFT, i, site[i].L.as<double>(), site[i].L.as<double>(), 0, left[i], left[i + 1], false, 1,
           rprec);
  for (int i = L - 1; i >= 0; --i)
    renorm(DMRG_DIR_RIGHT, i, site[i].R.as<double>(), site[i].R.as<double>(), 0, right[i + 1], right[i], false, 1,
           rprec);
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

// Terms of H_eff on the dot (i, width) with operators X (left, base B_LOPS)
// and Z (right, base B_ROPS); the channel site operator is dressed on the
// side that needs fewer formed operators.
std::vector<STerm> sigma_terms(Ctx& x, int i, int width, const OpSet& X, const OpSet& Z, Pool& pool,
                               LinCombBuilder& form, bool& left_dressed) {
  const SiteOp& W = x.H->site_op(i, width, x.H->mode_left(i), x.H->mode_right(i + width));
  const BondChannels& B0 = x.H->left_channels(i);
  const BondChannels& B1 = x.H->right_channels(i + width);
  std::vector<Group> GL = group_entries(W, true, -1), GR = group_entries(W, false, -1);
  auto prune = [&](std::vector<Group>& G, bool by_dst) {
    std::vector<Group> out;
    for (auto& g : G) {
      const int kk = by_dst ? Z.kind[g.key_ch] : X.kind[g.key_ch];
      if (kk == REF_ZERO) continue;
      std::vector<std::pair<int, double>> keep;
      for (auto& s : g.src) {
        const int sk = by_dst ? X.kind[s.first] : Z.kind[s.first];
        if (sk != REF_ZERO) keep.push_back(s);
      }
      if (keep.empty()) continue;
      g.src.swap(keep);
      out.push_back(std::move(g));
    }
    G.swap(out);
  };
  prune(GL, true);
  prune(GR, false);
  size_t fl = 0, fr = 0;
  for (auto& g : GL) fl += g.src.size() > 1;
  for (auto& g : GR) fr += g.src.size() > 1;
  left_dressed = fl <= fr;
  std::vector<STerm> terms;
  for (auto& g : left_dressed ? GL : GR) {
    const DotString& ds = x.H->dot_string(width, g.sid);
    STerm t{};
    t.sid = g.sid;
    if (left_dressed) {
      t.Z = Z.ref(g.key_ch, B_ROPS);
      t.pz = B1.ch[g.key_ch].parity;
      if (g.src.size() == 1) {
        t.X = X.ref(g.src[0].first, B_LOPS);
        t.alpha = g.src[0].second;
      } else {
        Sources ss;
        for (auto& s : g.src) ss.push_back({X.ref(s.first, B_LOPS), s.second});
        const Channel& ch = B1.ch[g.key_ch];
        t.X = pool.add(x.op_layout(i, ch.dna - ds.dna, ch.dnb - ds.dnb));
        emit_formation(form, t.X, ss);
        t.alpha = 1.0;
      }
    } else {
      t.X = X.ref(g.key_ch, B_LOPS);
      t.pz = B1.ch[g.src[0].first].parity;
      if (g.src.size() == 1) {
        t.Z = Z.ref(g.src[0].first, B_ROPS);
        t.alpha = g.src[0].second;
      } else {
        Sources ss;
        for (auto& s : g.src) ss.push_back({Z.ref(s.first, B_ROPS), s.second});
        const Channel& ch = B0.ch[g.key_ch];
        t.Z = pool.add(x.op_layout(i + width, ch.dna + ds.dna, ch.dnb + ds.dnb));
        emit_formation(form, t.Z, ss);
        t.alpha = 1.0;
      }
    }
    terms.push_back(t);
  }
  return terms;
}

inline int term_sign(const DotString& ds, const STerm& t, int nleft, int ndot) {
  int sgn = 1;
  if (((ds.parity + t.pz) & 1) && (nleft & 1)) sgn = -sgn;
  if (t.pz && (ndot & 1)) sgn = -sgn;
  return sgn;
}
}  // namespace

// left_first: only Z is batched (C and X shared), so stage 1 forms
// U = X C once and stage 2 multiplies U by each Z^T; otherwise stage 1 forms
// T = C Z^T and stage 2 applies X.
ContractionPlan& Ctx::sigma_plan(int i, int width, const OpSet& X, const OpSet& Z, bool left_first) {
  auto key = std::make_tuple(i, width, (X.first_order ? 1 : 0) + (left_first ? 2 : 0), Z.first_order ? 1 : 0);
  auto it = sigma_plans_.find(key);
  if (it != sigma_plans_.end()) return *it->second;
  return *(sigma_plans_[key] = make_sigma_plan(i, width, X, Z, left_first));
}

// As make_renorm_plan: no cache access, safe on the plan threads once the
// site layout and site operator of (i, width) exist.
std::unique_ptr<ContractionPlan> Ctx::make_sigma_plan(int i, int width, const OpSet& X, const OpSet& Z,
                                                      bool left_first) {
  auto P = std::make_unique<ContractionPlan>();
  P->left_first = left_first;
  const SiteLayout& S = layout(i, width);
  const Bond& bl = bonds[i];
  const Bond& br = bonds[i + width];
  Pool pool{B_DRESS};
  LinCombBuilder form;
  bool ld = true;
  std::vector<STerm> terms = sigma_terms(*this, i, width, X, Z, pool, form, ld);
  form.finish(*this, P->form);
  P->dressed_per_vec = pool.size;
  P->dress_left = ld;
  TwoStageBuilder TB;
  for (size_t b = 0; b < S.blk.size(); ++b)
    TB.outputs.push_back({long(S.blk[b].off), B_SOUT, S.blk[b].cols, S.blk[b].rows, S.blk[b].cols});
  for (auto& t : terms) {
    const DotString& ds = H->dot_string(width, t.sid);
    for (size_t e = 0; e < ds.val.size(); ++e) {
      const int n = ds.ket[e], np = ds.bra[e];
      const int nd = dot_qn(n, width).n();
      for (int a = 0; a < int(bl.q.size()); ++a) {
        const int b = S.find(a, n);
        if (b < 0) continue;
        const int c = S.blk[b].c;
        if (!has_blk(t.Z, c) || !has_blk(t.X, a)) continue;
        const int cp = opbra(t.Z, c), ap = opbra(t.X, a);
        const int bp = S.find(ap, np);
        if (bp < 0 || S.blk[bp].c != cp) continue;
        TwoStageBuilder::S2 s2{};
        s2.offC = long(S.blk[bp].off);
        s2.baseC = B_SOUT;
        s2.ldc = S.blk[bp].cols;
        s2.m = S.blk[bp].rows;
        s2.n = S.blk[bp].cols;
        GContrib g{};
        g.k = S.blk[b].rows;
        g.lda = S.blk[b].rows;
        g.alpha = t.alpha * ds.val[e] * term_sign(ds, t, bl.q[a].n(), nd);
        if (t.X.kind == REF_IDENTITY) {
          g.flags = GC_A_IDENTITY;
          g.baseA = B_LOPS;
        } else {
          g.offA = opoff(t.X, a);
          g.baseA = t.X.base;
        }
        if (t.Z.kind == REF_IDENTITY) {
          s2.t1 = -1;
          g.offB = long(S.blk[b].off);
          g.baseB = B_CIN;
          g.ldb = S.blk[b].cols;
        } else if (left_first) {
          // sigma(bp) += al U Z(c'<-c)^T with U = X(a'<-a) C(a,n,c) (m_a' x m_c)
          // (or C itself when X is the identity)
          g.k = S.blk[b].cols;
          g.offB = opoff(t.Z, c);
          g.baseB = t.Z.base;
          g.ldb = S.blk[b].cols;
          g.flags = GC_TRANS_B;
          if (t.X.kind == REF_IDENTITY) {
            s2.t1 = -1;
            g.offA = long(S.blk[b].off);
            g.baseA = B_CIN;
            g.lda = S.blk[b].cols;
          } else {
            auto tk = std::make_tuple(t.X.base, t.X.off, int(b));
            auto f = TB.t1_of.find(tk);
            if (f == TB.t1_of.end()) {
              TwoStageBuilder::T1 t1{};
              t1.merge = 1;  // X blocks share C: stack their rows
              t1.elems = long(bl.dim[ap]) * S.blk[b].cols;
              t1.job.ldc = S.blk[b].cols;
              t1.job.m = bl.dim[ap];
              t1.job.n = S.blk[b].cols;
              t1.con = {opoff(t.X, a), long(S.blk[b].off), S.blk[b].rows, S.blk[b].cols, S.blk[b].rows, 0, t.X.base,
                        B_CIN, 1.0};
              TB.t1.push_back(t1);
              f = TB.t1_of.emplace(tk, int(TB.t1.size()) - 1).first;
            }
            s2.t1 = f->second;
            s2.t_is_a = true;
            g.offA = 0;
            g.baseA = B_T;
            g.lda = S.blk[b].cols;
          }
        } else {
          auto tk = std::make_tuple(t.Z.base, t.Z.off, int(b));
          auto f = TB.t1_of.find(tk);
          if (f == TB.t1_of.end()) {
            // T(Z, a, n, c) = C(a,n,c) Z(c'<-c)^T  (m_a x m_c')
            TwoStageBuilder::T1 t1{};
            t1.merge = 2;  // the Z blocks share C: their products side by side
            t1.elems = long(S.blk[b].rows) * br.dim[cp];
            t1.job.ldc = br.dim[cp];
            t1.job.m = S.blk[b].rows;
            t1.job.n = br.dim[cp];
            t1.con = {long(S.blk[b].off), opoff(t.Z, c), S.blk[b].cols, S.blk[b].cols, S.blk[b].cols, GC_TRANS_B,
                      B_CIN, t.Z.base, 1.0};
            TB.t1.push_back(t1);
            f = TB.t1_of.emplace(tk, int(TB.t1.size()) - 1).first;
          }
          s2.t1 = f->second;
          g.offB = 0;
          g.baseB = B_T;
          g.ldb = br.dim[cp];
        }
        s2.con = g;
        TB.s2.push_back(s2);
      }
    }
  }
  finish_two_stage(*this, TB, P->main, true);
  if (std::getenv("DMRG_PLAN_STATS")) print_plan_stats("sigma", i, width, *P);
  return P;
}

void Ctx::parallel_for(int n, const std::function<void(int)>& fn) {
  std::vector<std::exception_ptr> err(n);
  std::atomic<int> next{0};
  auto work = [&]() {
    if (hipSetDevice(device) != hipSuccess) (void)hipGetLastError();
    for (int t = next++; t < n; t = next++) {
      try {
        fn(t);
      } catch (...) {
        err[t] = std::current_exception();
      }
    }
  };
  const int nth = std::max(1, std::min(plan_threads(), n));
  std::vector<std::thread> pool;
  for (int k = 1; k < nth; ++k) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

std::vector<std::unique_ptr<ContractionPlan>> Ctx::build_parallel(
    const std::vector<std::function<std::unique_ptr<ContractionPlan>()>>& fns) {
  const int n = int(fns.size());
  std::vector<std::unique_ptr<ContractionPlan>> built(n);
  std::vector<std::exception_ptr> err(n);
  std::atomic<int> next{0};
  std::vector<double> ms(n, 0.0);
  auto work = [&]() {
    // the current device is per host thread
    if (hipSetDevice(device) != hipSuccess) (void)hipGetLastError();
    for (int t = next++; t < n; t = next++) {
      const auto t0 = std::chrono::steady_clock::now();
      try {
        built[t] = fns[t]();
      } catch (...) {
        err[t] = std::current_exception();
      }
      ms[t] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
  };
  const int nth = std::max(1, std::min(plan_threads(), n));
  std::vector<std::thread> pool;
  for (int k = 1; k < nth; ++k) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  if (std::getenv("DMRG_PLAN_TIMING")) {
    double sum = 0, mx = 0;
    for (double v : ms) {
      sum += v;
      mx = std::max(mx, v);
    }
    std::fprintf(stderr, "[plan] %d plans on %d threads: %.1f ms of plan work, longest %.1f ms\n", n, nth, sum, mx);
  }
  return built;
}

// All plans of the DMRG-TDA sweeps (Fig. alg:dmrgtda) built up front on the
// plan threads: per site the two first-order renormalizations of each sweep
// direction (eqs. lopr1st, ropr1st) and the three sigmas (first-order left
// part, zeroth order, first-order right part), against layout-only
// first-order sets (their layouts depend only on bond and side).
void Ctx::prebuild_tda_plans() {
  std::vector<OpSet> fl(L + 1), fr(L + 1);
  for (int b = 0; b <= L; ++b) {
    alloc_opset(fl[b], b, 0, 0, true);
    alloc_opset(fr[b], b, 1, 0, true);
  }
  for (int i = 0; i < L; ++i) layout(i, 1);
  parallel_for(3 * L, [&](int t) {
    const int i = t / 3, k = t % 3;
    if (k == 0) H->site_op(i, 1, H->mode_left(i), H->mode_left(i + 1));
    else if (k == 1) H->site_op(i, 1, H->mode_right(i), H->mode_right(i + 1));
    else H->site_op(i, 1, H->mode_left(i), H->mode_right(i + 1));
  });
  typedef std::tuple<int, int, int, int> Key;
  std::vector<std::function<std::unique_ptr<ContractionPlan>()>> fns;
  std::vector<std::pair<int, Key>> dest;  // 0: renorm cache, 1: sigma cache
  auto add_r = [&](int dir, int i, const OpSet& src, const OpSet& dst, bool bf) {
    const Key k(dir, i, src.first_order ? 1 : 0, bf ? 1 : 0);
    if (renorm_plans_.count(k)) return;
    fns.push_back([this, dir, i, &src, &dst, bf]() { return make_renorm_plan(dir, i, src, dst, bf); });
    dest.push_back({0, k});
  };
  auto add_s = [&](int i, const OpSet& X, const OpSet& Z, bool lf) {
    const Key k(i, 1, (X.first_order ? 1 : 0) + (lf ? 2 : 0), Z.first_order ? 1 : 0);
    if (sigma_plans_.count(k)) return;
    fns.push_back([this, i, &X, &Z, lf]() { return make_sigma_plan(i, 1, X, Z, lf); });
    dest.push_back({1, k});
  };
  for (int i = 0; i < L; ++i) {
    add_s(i, fl[i], right[i + 1], false);
    add_s(i, left[i], right[i + 1], false);
    add_s(i, left[i], fr[i + 1], true);
    if (i + 1 < L) {
      add_r(DMRG_DIR_LEFT, i, fl[i], fl[i + 1], false);
      add_r(DMRG_DIR_LEFT, i, left[i], fl[i + 1], true);
    }
    if (i > 0) {
      add_r(DMRG_DIR_RIGHT, i, fr[i + 1], fr[i], false);
      add_r(DMRG_DIR_RIGHT, i, right[i + 1], fr[i], true);
    }
  }
  auto built = build_parallel(fns);
  for (size_t t = 0; t < built.size(); ++t) {
    if (dest[t].first == 0) renorm_plans_[dest[t].second] = std::move(built[t]);
    else sigma_plans_[dest[t].second] = std::move(built[t]);
  }
}

float* Ctx::f32_data(const OpSet& S) {
  if (S.f32) return S.data.as<float>();
  ensure_f32(S);
  return S.data32.as<float>();
}

void Ctx::ensure_f32(const OpSet& S) {
  OpSet& M = const_cast<OpSet&>(S);
  DMRG_REQUIRE(!M.f32, DMRG_ERR_INTERNAL, "operator set already held in FP32");
  if (M.f32_valid) return;
  const long n = long(M.per_vec) * M.nvec;
  M.data32.ensure(this, std::max<size_t>(size_t(n), 1) * 4);
  launch_convert_f64_f32(M.ptr(), M.data32.as<float>(), n, stream);
  DMRG_HIP(hipGetLastError());
  M.f32_valid = true;
}

void Ctx::sigma_general(int i, int width, const OpSet& X, const OpSet& Z, const double* C, long cstride, double* Sv,
                        long sstride, int batch, int prec) {
  const bool xb = X.nvec > 1, zb = Z.nvec > 1, cb = cstride != 0;
  ContractionPlan& P = sigma_plan(i, width, X, Z, zb && !xb && !cb && batch > 1);
  const bool dress_b = P.dress_left ? xb : zb;
  // stage-1 products: C Z^T depend on C and Z, X C (left first) on X and C
  const bool t_b = P.left_first ? (cb || xb) : (cb || zb);
  const size_t esz = prec == DMRG_FP64 ? 8 : 4;
  Bases b{};
  b.stride[B_CIN] = cstride;
  b.p[B_SOUT] = Sv;
  b.stride[B_SOUT] = sstride;
  b.stride[B_LOPS] = xb ? X.per_vec : 0;
  b.stride[B_ROPS] = zb ? Z.per_vec : 0;
  b.p[B_DRESS] = static_cast<double*>(
      workspace(WS_DRESS, ws_dress, std::max<size_t>(size_t(P.dressed_per_vec) * (dress_b ? batch : 1), 1) * esz));
  b.stride[B_DRESS] = dress_b ? P.dressed_per_vec : 0;
  b.p[B_T] = static_cast<double*>(
      workspace(WS_T, ws_T, std::max<size_t>(size_t(P.main.t_per_vec) * (t_b ? batch : 1), 1) * esz));
  b.stride[B_T] = t_b ? P.main.t_per_vec : 0;
  if (prec == DMRG_FP64) {
    DMRG_REQUIRE(!X.f32 && !Z.f32, DMRG_ERR_INTERNAL, "FP32 operator set in an FP64 sigma");
    b.p[B_CIN] = const_cast<double*>(C);
    b.p[B_LOPS] = X.ptr();
    b.p[B_ROPS] = Z.ptr();
    P.form.launch(*this, b, dress_b ? batch : 1, 0);
    for (auto& ch : P.main.chunks) {
      ch.first.launch(*this, b, t_b ? batch : 1, 0);
      ch.second.launch(*this, b, batch, 0, true, nullptr, 1);
    }
  } else {
    float* x32 = f32_data(X);
    float* z32 = f32_data(Z);
    const long cs = layout(i, width).size;
    const long nc = cb ? cs * batch : cs;
    float* c32 = static_cast<float*>(workspace(WS_C32, ws_c32, std::max<size_t>(size_t(nc), 1) * 4));
    launch_convert_f64_f32(C, c32, nc, stream);
    b.p[B_CIN] = reinterpret_cast<double*>(c32);
    b.stride[B_CIN] = cb ? cs : 0;
    b.p[B_LOPS] = reinterpret_cast<double*>(x32);
    b.p[B_ROPS] = reinterpret_cast<double*>(z32);
    P.form.launch(*this, b, dress_b ? batch : 1, prec);
    for (auto& ch : P.main.chunks) {
      ch.first.launch(*this, b, t_b ? batch : 1, prec, false, nullptr);
      ch.second.launch(*this, b, batch, prec, true, &b, 1);
    }
  }
  stats.sigma_flops = P.main.flops1 * (t_b ? batch : 1) + P.main.flops2 * batch;
  stats.sigma_main_flops = P.main.flops2 * batch;
  // stage-2 operand bytes: operators once, products and results per entry
  double by = 0;
  for (auto& ch : P.main.chunks) {
    const GemmPlan& G = ch.second;
    by += G.elems_a * esz * (dress_b ? batch : 1) + G.elems_b * esz * batch + G.elems_c * 8.0 * batch * 2;
  }
  stats.sigma_main_bytes = by;
}

void Ctx::sigma(int i, int width, int nvec, const double* Cin, double* Sout, int prec) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(nvec >= 1 && Cin && Sout, DMRG_ERR_INVALID_ARG, "bad sigma arguments");
  const SiteLayout& S = layout(i, width);
  sigma_plan(i, width, left[i], right[i + width]);  // plan outside the timed region
  ws_need_ = WsNeed();
  timed_sigma([&] {
    sigma_general(i, width, left[i], right[i + width], Cin, long(S.size), Sout, long(S.size), nvec, prec);
  });
  // workspace of this sigma, for a later no-allocation call with the same shape
  WsNeed& w = sigma_need_[std::make_tuple(i, width, nvec, prec)];
  double total = 0;
  for (int k = 0; k < WS_NSLOTS; ++k) {
    w.bytes[k] = std::max(w.bytes[k], ws_need_.bytes[k]);
    total += double((w.bytes[k] + 255) / 256 * 256);
  }
  stats.sigma_workspace_bytes = total;
}

void Ctx::release_workspaces() {
  sync();
  for (DBuf* b : {&ws_T, &ws_dress, &ws_blk, &ws_aux, &ws_c32, &ws_part, &ws_a32, &ws_fo, &ws_tda}) b->release();
  // The tile lists cached per (fold, batch size, shape) are many small
  // long-lived device buffers; kept after a sweep run they pin the large
  // segments that the run's transient buffers shared in a caching
  // allocator (measured: 19.9 GiB of lists holding 188 GiB reserved after a
  // response run), so they are rebuilt on demand instead.
  for (auto* cache : {&renorm_plans_, &sigma_plans_})
    for (auto& kv : *cache)
      for (auto& ch : kv.second->main.chunks) {
        ch.first.fold_tiles.clear();
        ch.second.fold_tiles.clear();
      }
}

void* Ctx::workspace(int slot, DBuf& buf, size_t bytes) {
  ws_need_.bytes[slot] = std::max(ws_need_.bytes[slot], bytes);
  if (no_alloc_) {
    DMRG_REQUIRE(bytes <= carve_len_[slot], DMRG_ERR_INTERNAL, "workspace beyond the size recorded for it");
    return static_cast<char*>(scratch_) + carve_off_[slot];
  }
  buf.ensure(this, bytes);
  return buf.p;
}

// The zeroth-order sigma of dmrg_sigma with every workspace in fixed regions
// of the static scratch (sizes recorded by an earlier dmrg_sigma of the same
// shape); no device memory is allocated or freed and no event is created.
// Nothing in the scratch needs clearing: every product, dressed operator,
// partial tile and FP32 vector is written before it is read.
void Ctx::sigma_noalloc(int i, int width, int nvec, const double* Cin, double* Sout, int prec) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(nvec >= 1 && Cin && Sout, DMRG_ERR_INVALID_ARG, "bad sigma arguments");
  DMRG_REQUIRE(scratch_, DMRG_ERR_STATE, "no scratch address for this device");
  const auto it = sigma_need_.find(std::make_tuple(i, width, nvec, prec));
  DMRG_REQUIRE(it != sigma_need_.end(), DMRG_ERR_STATE,
               "dmrg_sigma_noalloc needs one dmrg_sigma call with the same site, kind, nvec and precision "
               "first (it builds the plans and records the workspace sizes)");
  size_t off = 0;
  for (int k = 0; k < WS_NSLOTS; ++k) {
    carve_off_[k] = off;
    carve_len_[k] = it->second.bytes[k];
    off += (it->second.bytes[k] + 255) / 256 * 256;
  }
  DMRG_REQUIRE(off <= scratch_bytes(), DMRG_ERR_INVALID_ARG,
               "this sigma needs " + std::to_string(off) + " bytes of workspace, more than the " +
                   std::to_string(scratch_bytes()) + " bytes of the no-allocation scratch");
  const long n = long(layout(i, width).size);
  no_alloc_ = true;
  try {
    sigma_general(i, width, left[i], right[i + width], Cin, n, Sout, n, nvec, prec);
  } catch (...) {
    no_alloc_ = false;
    throw;
  }
  no_alloc_ = false;
  DMRG_HIP(hipGetLastError());
}

void Ctx::autotune(int i, int nvec, int prec, int* shapes, double* best_ms) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  DMRG_REQUIRE(i >= 0 && i < L && nvec >= 1, DMRG_ERR_INVALID_ARG, "bad autotune arguments");
  DMRG_REQUIRE(prec >= 0 && prec <= 2, DMRG_ERR_INVALID_ARG, "unsupported precision");
  const long n = long(layout(i, 1).size);
  DBuf cin, sout;
  cin.alloc(this, size_t(n) * nvec * 8);
  sout.alloc(this, size_t(n) * nvec * 8);
  // inputs: copies of the site's coefficient tensor when it has the current
  // layout's size, else a constant vector (timing only)
  if (site[i].C.p && site[i].C.bytes >= size_t(n) * 8) {
    for (int v = 0; v < nvec; ++v)
      DMRG_HIP(hipMemcpyAsync(cin.as<double>() + long(v) * n, site[i].C.as<double>(), size_t(n) * 8,
                              hipMemcpyDeviceToDevice, stream));
  } else {
    launch_fill_f64(cin.as<double>(), n * nvec, 1.0 / std::sqrt(double(std::max(n, 1L))), stream);
  }
  std::vector<int> cand = {-1, TILE_64x64, TILE_128x64, TILE_64x128};
  if (prec != DMRG_FP64) cand.push_back(TILE_128x128);
  int keep[2][3];
  for (int r = 0; r < 2; ++r)
    for (int f = 0; f < 3; ++f) keep[r][f] = tile_policy[prec][r][f];
  // device time of the sigma under one pair of shapes (warm-up call first:
  // tile lists and FP32 copies), best of three
  auto time_pair = [&](int s1, int s2) {
    for (int f = 0; f < 3; ++f) {
      tile_policy[prec][0][f] = s1;
      tile_policy[prec][1][f] = s2;
    }
    sigma(i, 1, nvec, cin.as<double>(), sout.as<double>(), prec);
    double t = 1e300;
    for (int rep = 0; rep < 3; ++rep) {
      sigma(i, 1, nvec, cin.as<double>(), sout.as<double>(), prec);
      t = std::min(t, double(stats.sigma_ms));
    }
    return t;
  };
  // the planner's pair is timed before and after the others (its best time is
  // the reference); a pair replaces it only if it is at least 2% faster both
  // in the sweep and in a confirming run, so that timing noise cannot flip
  // the choice
  double ref = time_pair(-1, -1);
  double best = 1e300;
  int b1 = -1, b2 = -1;
  for (int s1 : cand)
    for (int s2 : cand) {
      if (s1 == -1 && s2 == -1) continue;
      const double t = time_pair(s1, s2);
      if (t < best) {
        best = t;
        b1 = s1;
        b2 = s2;
      }
    }
  ref = std::min(ref, time_pair(-1, -1));
  if (b1 != -1 || b2 != -1) {
    const double again = std::max(best, time_pair(b1, b2));
    if (again < 0.98 * ref) {
      best = again;
    } else {
      b1 = b2 = -1;
      best = ref;
    }
  } else {
    best = ref;
  }
  for (int r = 0; r < 2; ++r)
    for (int f = 0; f < 3; ++f) tile_policy[prec][r][f] = keep[r][f];
  for (int f = 0; f < 3; ++f) {
    tile_policy[prec][0][f] = b1;
    tile_policy[prec][1][f] = b2;
  }
  sync();
  shapes[0] = b1;
  shapes[1] = b2;
  *best_ms = best;
}

void Ctx::mark_main(bool begin) {
  if (!timing_main_) return;
  (void)begin;
  if (main_events_used_ == int(main_events_.size())) {
    hipEvent_t e;
    DMRG_HIP(hipEventCreate(&e));
    main_events_.push_back(e);
  }
  DMRG_HIP(hipEventRecord(main_events_[main_events_used_++], stream));
}

void Ctx::diag(int i, int width, double* out) {
  require_gpu();
  DMRG_REQUIRE(ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
  auto key = std::make_pair(i, width);
  auto it = diag_plans_.find(key);
  const SiteLayout& S = layout(i, width);
  if (it == diag_plans_.end()) {
    auto P = std::make_unique<DiagPlan>();
    Pool pool{B_DRESS};
    LinCombBuilder form;
    bool ld = true;
    std::vector<STerm> terms = sigma_terms(*this, i, width, left[i], right[i + width], pool, form, ld);
    form.finish(*this, P->form);
    P->dressed_per_vec = pool.size;
    const Bond& bl = bonds[i];
    std::vector<std::vector<DiagTerm>> per(S.blk.size());
    for (auto& t : terms) {
      if (t.X.kind == REF_OP && (t.X.lay->dna || t.X.lay->dnb)) continue;
      if (t.Z.kind == REF_OP && (t.Z.lay->dna || t.Z.lay->dnb)) continue;
      const DotString& ds = H->dot_string(width, t.sid);
      for (size_t e = 0; e < ds.val.size(); ++e) {
        if (ds.bra[e] != ds.ket[e]) continue;
        const int n = ds.ket[e];
        const int nd = dot_qn(n, width).n();
        for (int a = 0; a < int(bl.q.size()); ++a) {
          const int b = S.find(a, n);
          if (b < 0) continue;
          const int c = S.blk[b].c;
          if (!has_blk(t.X, a) || !has_blk(t.Z, c)) continue;
          DiagTerm d{};
          d.offX = t.X.kind == REF_IDENTITY ? -1 : opoff(t.X, a);
          d.baseX = t.X.kind == REF_IDENTITY ? 0 : t.X.base;
          d.offZ = t.Z.kind == REF_IDENTITY ? -1 : opoff(t.Z, c);
          d.baseZ = t.Z.kind == REF_IDENTITY ? 0 : t.Z.base;
          d.alpha = t.alpha * ds.val[e] * term_sign(ds, t, bl.q[a].n(), nd);
          per[b].push_back(d);
        }
      }
    }
    std::vector<DiagJob> jobs;
    std::vector<DiagTerm> dt;
    for (size_t b = 0; b < S.blk.size(); ++b) {
      jobs.push_back({long(S.blk[b].off), B_SOUT, S.blk[b].rows, S.blk[b].cols, int(dt.size()), 0, 0});
      dt.insert(dt.end(), per[b].begin(), per[b].end());
      jobs.back().t1 = int(dt.size());
    }
    upload(*this, P->jobs, jobs);
    upload(*this, P->terms, dt);
    P->njobs = int(jobs.size());
    it = diag_plans_.emplace(key, std::move(P)).first;
  }
  DiagPlan& P = *it->second;
  Bases b{};
  b.p[B_LOPS] = left[i].ptr();
  b.p[B_ROPS] = right[i + width].ptr();
  b.p[B_SOUT] = out;
  ws_dress.ensure(this, std::max<size_t>(size_t(P.dressed_per_vec), 1) * 8);
  b.p[B_DRESS] = ws_dress.as<double>();
  P.form.launch(*this, b, 1);
  launch_diag_jobs_f64(P.jobs.as<DiagJob>(), P.njobs, P.terms.as<DiagTerm>(), b, stream);
  DMRG_HIP(hipGetLastError());
}

}  // namespace dmrg
