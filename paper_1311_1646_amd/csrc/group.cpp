// Grouped sigma of many independent problems (the many-instance regime of
// small DMRG problems): the zeroth-order one-site sigma (Sec. III B, eq.
// hzero_sb) of every member context at its own site, as one launch per
// stage for all members.
//
// Each member keeps its own cached plan (work lists relative to base slots).
// The group concatenates those lists into one list per stage, every job and
// formation group tagged with its member's index, and the kernels take the
// member's base table from a device array of tables.  A step is then: one
// FP64 -> FP32 conversion of all inputs (FP32 contractions), one formation of
// the dressed operators, and per workspace chunk one products launch, one
// accumulation launch and (for split contribution lists) one reduction.  The
// step can be captured once into a HIP graph and replayed; the graph reads
// the base tables from device memory, so new input / output buffers only
// re-upload the tables.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "engine.hpp"
#include "kernels_mfma.hpp"

namespace dmrg {

namespace {

template <class T>
std::vector<T> download(const DBuf& b, size_t n) {
  std::vector<T> v(n);
  if (n) DMRG_HIP(hipMemcpy(v.data(), b.p, n * sizeof(T), hipMemcpyDeviceToHost));
  return v;
}

template <class T>
void upload_to(Ctx& x, DBuf& buf, const std::vector<T>& v) {
  buf.alloc(&x, std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty()) DMRG_HIP(hipMemcpy(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

}  // namespace

class SigmaGroup {
 public:
  SigmaGroup(const std::vector<Ctx*>& xs, const std::vector<int>& sites, int nvec, int prec);
  ~SigmaGroup();
  void sigma(const double* const* C, double* const* S, const size_t* lens, bool use_graph);
  std::string err;
  double flops = 0, ms = 0;
  int launches = 0, graph_nodes = 0;

 private:
  std::vector<Ctx*> x_;
  std::vector<int> site_;
  std::vector<unsigned long> gen_;
  std::vector<long> size_;
  int nvec_, prec_;
  std::vector<ContractionPlan*> plan_;
  std::vector<DBuf> dress_, t_, c32_;  // per-member workspaces (owned by the group)
  std::vector<Bases> bases_;           // per-member base tables (host copy)
  DBuf ib_, conv_, part_;              // device tables and partial tiles
  std::vector<ConvJob> convs_;
  long conv_max_ = 0;
  LinCombPlan form_;
  std::vector<std::pair<GemmPlan, GemmPlan>> chunks_;
  Bases tmpl_{};  // base table of member 0 (decides the batch folding)
  std::vector<const double*> last_c_;
  std::vector<double*> last_s_;
  hipStream_t gs_ = nullptr;
  hipEvent_t ev_in_ = nullptr, ev_out_ = nullptr, t0_ = nullptr, t1_ = nullptr;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  bool warm_ = false;

  Ctx& x0() { return *x_[0]; }
  void merge_form();
  void merge_gemm(GemmPlan& out, bool stage2, int chunk);
  void set_tables(const double* const* C, double* const* S);
  int enqueue(hipStream_t s);  // the step's launches; returns their count
  void launch_gemm(const GemmPlan& P, int role, bool out_f64, hipStream_t s, int& n);
};

SigmaGroup::SigmaGroup(const std::vector<Ctx*>& xs, const std::vector<int>& sites, int nvec, int prec)
    : x_(xs), site_(sites), nvec_(nvec), prec_(prec) {
  DMRG_REQUIRE(!x_.empty() && x_.size() == site_.size(), DMRG_ERR_INVALID_ARG, "need one site per context");
  DMRG_REQUIRE(nvec >= 1, DMRG_ERR_INVALID_ARG, "nvec must be >= 1");
  DMRG_REQUIRE(prec == DMRG_FP64 || prec == DMRG_FP32 || prec == DMRG_BF16X3, DMRG_ERR_INVALID_ARG,
               "unsupported precision");
  const int n = int(x_.size());
  for (int i = 0; i < n; ++i) {
    Ctx& x = *x_[i];
    x.require_gpu();
    DMRG_REQUIRE(x.device == x0().device && x.stream == x0().stream, DMRG_ERR_INVALID_ARG,
                 "grouped contexts must share the device and the stream");
    DMRG_REQUIRE(x.ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops on every grouped context first");
    DMRG_REQUIRE(site_[i] >= 0 && site_[i] < x.L, DMRG_ERR_INVALID_ARG, "bad site");
  }
  DMRG_HIP(hipSetDevice(x0().device));
  const size_t esz = prec == DMRG_FP64 ? 8 : 4;
  plan_.resize(n);
  dress_.resize(n);
  t_.resize(n);
  c32_.resize(n);
  bases_.assign(n, Bases{});
  gen_.resize(n);
  size_.resize(n);
  for (int i = 0; i < n; ++i) {
    Ctx& x = *x_[i];
    const int s = site_[i];
    gen_[i] = x.generation;
    size_[i] = long(x.layout(s, 1).size);
    plan_[i] = &x.sigma_plan(s, 1, x.left[s], x.right[s + 1]);
    const ContractionPlan& P = *plan_[i];
    dress_[i].alloc(&x, std::max<size_t>(size_t(P.dressed_per_vec), 1) * esz);
    t_[i].alloc(&x, std::max<size_t>(size_t(P.main.t_per_vec) * nvec, 1) * esz);
    Bases& b = bases_[i];
    b.stride[B_CIN] = size_[i];
    b.stride[B_SOUT] = size_[i];
    b.p[B_DRESS] = dress_[i].as<double>();
    b.p[B_T] = t_[i].as<double>();
    b.stride[B_T] = P.main.t_per_vec;
    if (prec == DMRG_FP64) {
      b.p[B_LOPS] = x.left[s].ptr();
      b.p[B_ROPS] = x.right[s + 1].ptr();
    } else {
      c32_[i].alloc(&x, std::max<size_t>(size_t(size_[i]) * nvec, 1) * 4);
      b.p[B_CIN] = reinterpret_cast<double*>(c32_[i].as<float>());
      b.p[B_LOPS] = reinterpret_cast<double*>(x.f32_data(x.left[s]));
      b.p[B_ROPS] = reinterpret_cast<double*>(x.f32_data(x.right[s + 1]));
      conv_max_ = std::max(conv_max_, size_[i] * nvec);
    }
  }
  tmpl_ = bases_[0];
  merge_form();
  size_t nch = 0;
  for (auto* P : plan_) nch = std::max(nch, P->main.chunks.size());
  chunks_.resize(nch);
  for (size_t c = 0; c < nch; ++c) {
    merge_gemm(chunks_[c].first, false, int(c));
    merge_gemm(chunks_[c].second, true, int(c));
  }
  ib_.alloc(&x0(), sizeof(Bases) * n);
  if (prec != DMRG_FP64) conv_.alloc(&x0(), sizeof(ConvJob) * n);
  DMRG_HIP(hipStreamCreateWithFlags(&gs_, hipStreamNonBlocking));
  for (hipEvent_t* e : {&ev_in_, &ev_out_}) DMRG_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  DMRG_HIP(hipEventCreate(&t0_));
  DMRG_HIP(hipEventCreate(&t1_));
  for (int i = 0; i < n; ++i)
    flops += plan_[i]->main.flops1 * nvec + plan_[i]->main.flops2 * nvec;
}

SigmaGroup::~SigmaGroup() {
  if (exec_) (void)hipGraphExecDestroy(exec_);
  if (graph_) (void)hipGraphDestroy(graph_);
  for (hipEvent_t e : {ev_in_, ev_out_, t0_, t1_})
    if (e) (void)hipEventDestroy(e);
  if (gs_) {
    (void)hipStreamSynchronize(gs_);
    (void)hipStreamDestroy(gs_);
  }
}

// Formation of the dressed operators of every member in one list: groups,
// targets, sources, coefficient rows and identity additions concatenated,
// each group and addition tagged with its member.
void SigmaGroup::merge_form() {
  std::vector<LCGroup> g;
  std::vector<LCTarget> t;
  std::vector<LCSource> u;
  std::vector<double> cf;
  std::vector<DiagAdd> d;
  long max_size = 0;
  for (size_t i = 0; i < plan_.size(); ++i) {
    const LinCombPlan& F = plan_[i]->form;
    auto gi = download<LCGroup>(F.g, F.ng);
    auto ti = download<LCTarget>(F.t, F.nt);
    int nu = 0;
    for (auto& q : gi) nu = std::max(nu, q.u1);
    auto ui = download<LCSource>(F.u, nu);
    auto ci = download<double>(F.coef, size_t(nu) * kLCGroup);
    auto di = download<DiagAdd>(F.d, F.nd);
    const int t_off = int(t.size()), u_off = int(u.size());
    for (auto q : gi) {
      q.t0 += t_off;
      q.u0 += u_off;
      q.u1 += u_off;
      q.inst = int(i);
      g.push_back(q);
    }
    t.insert(t.end(), ti.begin(), ti.end());
    u.insert(u.end(), ui.begin(), ui.end());
    cf.insert(cf.end(), ci.begin(), ci.end());
    for (auto q : di) {
      q.inst = int(i);
      d.push_back(q);
    }
    max_size = std::max(max_size, F.max_size);
  }
  upload_to(x0(), form_.g, g);
  upload_to(x0(), form_.t, t);
  upload_to(x0(), form_.u, u);
  upload_to(x0(), form_.coef, cf);
  upload_to(x0(), form_.coef32, std::vector<float>(cf.begin(), cf.end()));
  upload_to(x0(), form_.d, d);
  form_.ng = int(g.size());
  form_.nt = int(t.size());
  form_.nd = int(d.size());
  form_.max_size = max_size;
}

// One stage of one workspace chunk for every member that has that chunk:
// jobs (tagged with the member), their contributions and gather entries.
void SigmaGroup::merge_gemm(GemmPlan& out, bool stage2, int chunk) {
  std::vector<GJob> jobs;
  std::vector<std::vector<GContrib>> per;
  std::vector<int> gather;
  for (size_t i = 0; i < plan_.size(); ++i) {
    const auto& ch = plan_[i]->main.chunks;
    if (chunk >= int(ch.size())) continue;
    const GemmPlan& P = stage2 ? ch[chunk].second : ch[chunk].first;
    const size_t nj = P.shapes.size();
    if (nj == 0) continue;
    auto ji = download<GJob>(P.jobs, nj);
    auto ci = download<GContrib>(P.con, size_t(P.ncon));
    size_t ng = 0;
    for (auto& j : ji)
      if (j.flags & (GJ_GATHER_A | GJ_GATHER_B))
        ng = std::max(ng, size_t(j.pad) + size_t((j.flags & GJ_GATHER_A) ? j.m : j.n));
    auto gi = download<int>(P.gat, ng);
    const int g_off = int(gather.size());
    for (auto j : ji) {
      per.emplace_back(ci.begin() + j.c0, ci.begin() + j.c1);
      if (j.flags & (GJ_GATHER_A | GJ_GATHER_B)) j.pad += g_off;
      j.inst = int(i);
      jobs.push_back(j);
    }
    gather.insert(gather.end(), gi.begin(), gi.end());
  }
  build_gemm_plan(x0(), out, jobs, per, gather);
}

void SigmaGroup::set_tables(const double* const* C, double* const* S) {
  const int n = int(x_.size());
  convs_.clear();
  for (int i = 0; i < n; ++i) {
    DMRG_REQUIRE(C[i] && S[i], DMRG_ERR_INVALID_ARG, "null member vectors");
    if (prec_ == DMRG_FP64) bases_[i].p[B_CIN] = const_cast<double*>(C[i]);
    else convs_.push_back({C[i], c32_[i].as<float>(), size_[i] * nvec_});
    bases_[i].p[B_SOUT] = S[i];
  }
  // the previous step may still read the tables
  DMRG_HIP(hipStreamSynchronize(gs_));
  DMRG_HIP(hipStreamSynchronize(x0().stream));
  DMRG_HIP(hipMemcpy(ib_.p, bases_.data(), sizeof(Bases) * n, hipMemcpyHostToDevice));
  if (!convs_.empty())
    DMRG_HIP(hipMemcpy(conv_.p, convs_.data(), sizeof(ConvJob) * convs_.size(), hipMemcpyHostToDevice));
  last_c_.assign(C, C + n);
  last_s_.assign(S, S + n);
}

void SigmaGroup::launch_gemm(const GemmPlan& P, int role, bool out_f64, hipStream_t s, int& n) {
  if (P.ntiles == 0) return;
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
  if (nvec_ > 1 && batched(tmpl_, P.mask_c, true)) {
    if (!batched(tmpl_, P.mask_a, false) && batched(tmpl_, P.mask_b, true)) fold = FOLD_N;
    else if (!batched(tmpl_, P.mask_b, false) && (P.mask_a == 0 || batched(tmpl_, P.mask_a, true))) fold = FOLD_M;
  }
  int want = x0().tile_policy[prec_][role][fold];
  if (prec_ == DMRG_FP64 && want == TILE_128x128) want = TILE_64x64;
  const GemmPlan::FoldTiles& F = P.fold_lists(x0(), fold, nvec_, want);
  void* part = nullptr;
  if (F.nslots > 0) {
    const size_t esz = prec_ == DMRG_FP64 ? 8 : 4;
    const size_t bytes =
        size_t(F.nslots) * (fold == FOLD_NONE ? nvec_ : 1) * size_t(tile_rows(F.shape)) * tile_cols(F.shape) * esz;
    if (part_.bytes < bytes) part_.alloc(&x0(), bytes);
    part = part_.p;
  }
  const Bases* ib = ib_.as<Bases>();
  if (prec_ == DMRG_FP64 && !x0().fp64_mfma)
    throw Error(DMRG_ERR_INVALID_ARG, "grouped FP64 sigma needs the matrix-core kernel (DMRG_FP64_GEMM unset)");
  launch_grouped_gemm(prec_, out_f64, role, F.shape, F.tiles.as<GTile>(), F.ntiles, P.jobs.as<GJob>(),
                      P.con.as<GContrib>(), P.gat.as<int>(), F.segs.as<GSeg>(), F.nslots, part, tmpl_, tmpl_, fold,
                      nvec_, s, ib);
  ++n;
  if (F.nred > 0) {
    launch_reduce_partials(prec_, out_f64, F.shape, F.red.as<GRed>(), F.nred, P.jobs.as<GJob>(), F.nslots, part,
                           tmpl_, fold, nvec_, s, ib);
    ++n;
  }
}

int SigmaGroup::enqueue(hipStream_t s) {
  int n = 0;
  const Bases* ib = ib_.as<Bases>();
  if (prec_ != DMRG_FP64) {
    launch_convert_list(conv_.as<ConvJob>(), int(convs_.size()), conv_max_, s);
    ++n;
  }
  if (form_.ng) {
    launch_lincomb_grouped(prec_, form_.g.as<LCGroup>(), form_.ng, form_.t.as<LCTarget>(), form_.u.as<LCSource>(),
                           form_.coef.as<double>(), form_.coef32.as<float>(), form_.max_size, tmpl_, 1, s, ib);
    ++n;
  }
  if (form_.nd) {
    if (prec_ == DMRG_FP64) launch_diag_add_f64(form_.d.as<DiagAdd>(), form_.nd, tmpl_, 1, s, ib);
    else launch_diag_add_f32(form_.d.as<DiagAdd>(), form_.nd, tmpl_, 1, s, ib);
    ++n;
  }
  for (auto& ch : chunks_) {
    launch_gemm(ch.first, 0, prec_ == DMRG_FP64, s, n);
    launch_gemm(ch.second, 1, true, s, n);
  }
  DMRG_HIP(hipGetLastError());
  return n;
}

void SigmaGroup::sigma(const double* const* C, double* const* S, const size_t* lens, bool use_graph) {
  const int n = int(x_.size());
  DMRG_REQUIRE(C && S && lens, DMRG_ERR_INVALID_ARG, "null arrays");
  for (int i = 0; i < n; ++i) {
    DMRG_REQUIRE(x_[i]->generation == gen_[i], DMRG_ERR_STATE,
                 "a grouped context changed its MPS or operators since the group was created");
    DMRG_REQUIRE(lens[i] == size_t(size_[i]) * nvec_, DMRG_ERR_INVALID_ARG, "len of a member is not nvec * size");
  }
  DMRG_HIP(hipSetDevice(x0().device));
  bool same = int(last_c_.size()) == n;
  for (int i = 0; same && i < n; ++i) same = last_c_[i] == C[i] && last_s_[i] == S[i];
  if (!same) set_tables(C, S);
  // inputs are produced on the members' stream; the step runs on the
  // group's stream and the members' stream waits for its end
  DMRG_HIP(hipEventRecord(ev_in_, x0().stream));
  DMRG_HIP(hipStreamWaitEvent(gs_, ev_in_, 0));
  DMRG_HIP(hipEventRecord(t0_, gs_));
  if (!use_graph || !warm_) {
    launches = enqueue(gs_);  // the first step builds the tile lists and partial buffers
    warm_ = true;
  } else {
    if (!exec_) {
      // capture: nothing may be allocated from here on
      for (Ctx* x : x_) x->no_alloc_ = true;
      DMRG_HIP(hipStreamBeginCapture(gs_, hipStreamCaptureModeThreadLocal));
      try {
        launches = enqueue(gs_);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(gs_, &g);
        if (g) (void)hipGraphDestroy(g);
        for (Ctx* x : x_) x->no_alloc_ = false;
        throw;
      }
      for (Ctx* x : x_) x->no_alloc_ = false;
      DMRG_HIP(hipStreamEndCapture(gs_, &graph_));
      size_t nodes = 0;
      DMRG_HIP(hipGraphGetNodes(graph_, nullptr, &nodes));
      graph_nodes = int(nodes);
      DMRG_HIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
      DMRG_HIP(hipEventRecord(t0_, gs_));
    }
    DMRG_HIP(hipGraphLaunch(exec_, gs_));
  }
  DMRG_HIP(hipEventRecord(t1_, gs_));
  DMRG_HIP(hipEventRecord(ev_out_, gs_));
  DMRG_HIP(hipStreamWaitEvent(x0().stream, ev_out_, 0));
  DMRG_HIP(hipEventSynchronize(t1_));
  float f = 0;
  DMRG_HIP(hipEventElapsedTime(&f, t0_, t1_));
  ms = f;
}

}  // namespace dmrg

// ---------------------------------------------------------------- C-ABI

struct dmrg_group {
  dmrg::SigmaGroup* g;
};

namespace {
thread_local std::string g_group_error;

template <class F>
int group_guard(dmrg_group* h, F&& f) {
  if (!h || !h->g) return DMRG_ERR_INVALID_ARG;
  try {
    h->g->err.clear();
    f(*h->g);
    return DMRG_OK;
  } catch (const dmrg::Error& e) {
    h->g->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    h->g->err = "host allocation failed";
    return DMRG_ERR_OOM;
  } catch (const std::exception& e) {
    h->g->err = e.what();
    return DMRG_ERR_INTERNAL;
  }
}
}  // namespace

extern "C" {

int dmrg_group_create(dmrg_ctx* const* ctxs, int n, const int* sites, int nvec, int prec, dmrg_group** out) {
  if (!out) return DMRG_ERR_INVALID_ARG;
  *out = nullptr;
  try {
    DMRG_REQUIRE(ctxs && sites && n >= 1, DMRG_ERR_INVALID_ARG, "need n >= 1 contexts and sites");
    std::vector<dmrg::Ctx*> xs;
    for (int i = 0; i < n; ++i) {
      DMRG_REQUIRE(ctxs[i] && ctxs[i]->x, DMRG_ERR_INVALID_ARG, "null context");
      xs.push_back(ctxs[i]->x);
    }
    *out = new dmrg_group{new dmrg::SigmaGroup(xs, std::vector<int>(sites, sites + n), nvec, prec)};
    return DMRG_OK;
  } catch (const dmrg::Error& e) {
    g_group_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_group_error = "host allocation failed";
    return DMRG_ERR_OOM;
  } catch (const std::exception& e) {
    g_group_error = e.what();
    return DMRG_ERR_INTERNAL;
  }
}

int dmrg_group_sigma(dmrg_group* g, const double* const* C_in, double* const* sigma_out, const size_t* lens,
                     int use_graph) {
  return group_guard(g, [&](dmrg::SigmaGroup& G) { G.sigma(C_in, sigma_out, lens, use_graph != 0); });
}

int dmrg_group_stats(dmrg_group* g, double* flops, double* ms, int* launches, int* graph_nodes) {
  return group_guard(g, [&](dmrg::SigmaGroup& G) {
    if (flops) *flops = G.flops;
    if (ms) *ms = G.ms;
    if (launches) *launches = G.launches;
    if (graph_nodes) *graph_nodes = G.graph_nodes;
  });
}

const char* dmrg_group_last_error(const dmrg_group* g) {
  if (!g || !g->g) return g_group_error.c_str();
  return g->g->err.c_str();
}

int dmrg_group_destroy(dmrg_group* g) {
  if (!g) return DMRG_ERR_INVALID_ARG;
  delete g->g;
  delete g;
  return DMRG_OK;
}

}  // extern "C"
