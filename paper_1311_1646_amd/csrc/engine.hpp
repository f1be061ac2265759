// Context, operator pools and the contraction planners (host side).
#pragma once
#include <map>
#include <memory>
#include <string>
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

// Reference to an operator (or the identity) at one bond.
struct ORef {
  const double* p = nullptr;
  const OpLayout* lay = nullptr;  // null = identity
  bool identity() const { return lay == nullptr; }
};

// Operators of one block at one bond: side 0 = left-block operators Lop_b[w],
// side 1 = right-block operators Rop_b[w], for every channel w of the bond.
struct OpClass {
  const OpLayout* lay = nullptr;
  int nslots = 0;
  DBuf data;
};
struct OpSet {
  int bond = -1, side = 0;
  bool valid = false;
  std::vector<int> cls, slot;  // per channel; cls -1 = identity channel
  std::vector<OpClass> classes;
  ORef ref(int w) const {
    ORef r;
    if (cls[w] < 0) return r;
    const OpClass& C = classes[cls[w]];
    r.lay = C.lay;
    r.p = C.data.as<double>() + size_t(slot[w]) * C.lay->size;
    return r;
  }
  size_t bytes() const {
    size_t b = 0;
    for (auto& c : classes) b += c.data.bytes;
    return b;
  }
};

// Scratch pool of extra operators (dressed operators, building blocks).
struct OpPool {
  int bond = -1;
  std::map<std::pair<int, int>, int> class_of;
  std::vector<OpClass> classes;
  struct Item { int cls, slot; };
  std::vector<Item> items;
  int add(const OpLayout* lay);  // returns item id (before allocate())
  void allocate(Ctx* c);
  ORef ref(int id) const {
    const OpClass& C = classes[items[id].cls];
    return ORef{C.data.as<double>() + size_t(items[id].slot) * C.lay->size, C.lay};
  }
};

// Device-side execution lists of one contraction step.
struct GemmList {
  std::vector<GJob> jobs;
  std::vector<std::vector<GContrib>> per_job;
  std::unordered_map<const void*, int> job_of;
  int job(void* C, int ldc, int m, int n, int flags);
  void add(int j, const GContrib& c) { per_job[j].push_back(c); }
  double flops(int batch) const;
  void run(Ctx& x, int batch, long sA, long sB, long sC);
  bool empty() const { return jobs.empty(); }
};

struct LinComb {
  std::vector<LCTarget> t;
  std::vector<LCSource> s;
  std::vector<DiagAdd> d;
  long max_size = 0;
  void target(double* out, long size, bool acc) {
    t.push_back({out, size, int(s.size()), int(s.size()), acc ? 1 : 0, 0});
    if (size > max_size) max_size = size;
  }
  void source(const double* p, double c) {
    s.push_back({p, c});
    t.back().s1 = int(s.size());
  }
  void run(Ctx& x, int batch, long stride);
};

struct SiteTensors {
  DBuf L, R, C;  // device FP64, flat one-site layout
};

class Ctx {
 public:
  Ctx(int L, int na, int nb, const double* h, const double* eri, double ecore, int device, void* stream,
      const dmrg_allocator* alloc);
  ~Ctx();

  int L, Na, Nb;
  int device;
  hipStream_t stream = nullptr;
  dmrg_allocator allocator{};
  std::string err;
  std::unique_ptr<QCHamiltonian> H;

  // MPS
  bool have_mps = false;
  std::vector<Bond> bonds;
  std::vector<std::vector<std::vector<double>>> lam;  // [bond][sector] host
  std::vector<SiteTensors> site;
  const SiteLayout& layout(int i, int width);
  const OpLayout* op_layout(int bond, int dna, int dnb);

  // zeroth-order operators
  std::vector<OpSet> left, right;  // left[b] = Lop_b, right[b] = Rop_b
  int ops_prec = -1;

  // stats
  dmrg_stats stats{};

  void* dev_alloc(size_t bytes);
  void dev_free(void* p);
  void require_gpu() const;

  void import_mps(const int* nsec, const int* sectors, const double* Ld, const double* Rd, const double* Cd,
                  const double* lam);
  void export_mps(int* nsec_out, int* sectors_out, double* Ld, double* Rd, double* Cd, double* lam_out,
                  size_t* sizes);
  void build_ops(int prec);
  void alloc_opset(OpSet& S, int bond, int side);
  // zeroth-order renormalization across one site
  void renorm_left(int i, const double* Abra, const double* Aket, const OpSet& src, OpSet& dst);
  void renorm_right(int i, const double* Abra, const double* Aket, const OpSet& src, OpSet& dst);
  void sigma(int i, int width, int nvec, const double* Cin, double* Sout);
  void diag(int i, int width, double* out);

 private:
  std::map<std::pair<int, int>, std::unique_ptr<SiteLayout>> layouts_;
  std::map<std::tuple<int, int, int>, std::unique_ptr<OpLayout>> op_layouts_;
};

}  // namespace dmrg
