// extern "C" entry points (see include/dmrg.h).
#include <cstring>
#include <new>
#include <string>

#include "engine.hpp"
#include "rpa_reduced.hpp"

namespace dmrg {
int debug_mpo_dense_left(QCHamiltonian& H, int wide_bond, double* out);
int debug_mpo_dense_right(QCHamiltonian& H, int wide_bond, double* out);
}  // namespace dmrg


namespace {
thread_local std::string g_create_error;

template <class F>
int guard(dmrg_ctx* c, F&& f) {
  if (!c || !c->x) return DMRG_ERR_INVALID_ARG;
  try {
    c->x->err.clear();
    f(*c->x);
    return DMRG_OK;
  } catch (const dmrg::Error& e) {
    c->x->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    c->x->err = "host allocation failed";
    return DMRG_ERR_OOM;
  } catch (const std::invalid_argument& e) {
    c->x->err = e.what();
    return DMRG_ERR_INVALID_ARG;
  } catch (const std::exception& e) {
    c->x->err = e.what();
    return DMRG_ERR_INTERNAL;
  }
}
}  // namespace

extern "C" {

int dmrg_create(int L, int n_alpha, int n_beta, const double* h, const double* eri, double ecore, int device,
                void* stream, const dmrg_allocator* alloc, dmrg_ctx** out) {
  if (!out) return DMRG_ERR_INVALID_ARG;
  *out = nullptr;
  try {
    auto* c = new dmrg_ctx{new dmrg::Ctx(L, n_alpha, n_beta, h, eri, ecore, device, stream, alloc)};
    *out = c;
    return DMRG_OK;
  } catch (const dmrg::Error& e) {
    g_create_error = e.what();
    return e.code;
  } catch (const std::invalid_argument& e) {
    g_create_error = e.what();
    return DMRG_ERR_INVALID_ARG;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    return DMRG_ERR_OOM;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return DMRG_ERR_INTERNAL;
  }
}

int dmrg_destroy(dmrg_ctx* ctx) {
  if (!ctx) return DMRG_ERR_INVALID_ARG;
  delete ctx->x;
  delete ctx;
  return DMRG_OK;
}

const char* dmrg_last_error(const dmrg_ctx* ctx) {
  if (!ctx || !ctx->x) return g_create_error.c_str();
  return ctx->x->err.c_str();
}

int dmrg_num_channels(dmrg_ctx* ctx, int bond, int* out) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(bond >= 0 && bond <= x.L && out, DMRG_ERR_INVALID_ARG, "bad bond");
    *out = int(x.H->left_channels(bond).ch.size());
  });
}

int dmrg_import_mps(dmrg_ctx* ctx, const int* nsec, const int* sectors, const double* Ldata, const double* Rdata,
                    const double* Cdata, const double* lam) {
  return guard(ctx, [&](dmrg::Ctx& x) { x.import_mps(nsec, sectors, Ldata, Rdata, Cdata, lam); });
}

int dmrg_export_mps(dmrg_ctx* ctx, int* nsec_out, int* sectors_out, double* Ldata, double* Rdata, double* Cdata,
                    double* lam, size_t* sizes_out) {
  return guard(ctx, [&](dmrg::Ctx& x) { x.export_mps(nsec_out, sectors_out, Ldata, Rdata, Cdata, lam, sizes_out); });
}

int dmrg_get_layout(dmrg_ctx* ctx, int site, int width, int* nblocks_out, int* blocks_out, size_t* size_out) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    const dmrg::SiteLayout& S = x.layout(site, width);
    if (nblocks_out) *nblocks_out = int(S.blk.size());
    if (size_out) *size_out = S.size;
    if (blocks_out)
      for (size_t b = 0; b < S.blk.size(); ++b) {
        int* o = blocks_out + 6 * b;
        o[0] = S.blk[b].a;
        o[1] = S.blk[b].n;
        o[2] = S.blk[b].c;
        o[3] = S.blk[b].rows;
        o[4] = S.blk[b].cols;
        o[5] = int(S.blk[b].off);
      }
  });
}

namespace {
bool valid_prec(int p) { return p == DMRG_FP64 || p == DMRG_FP32 || p == DMRG_BF16X3; }
}  // namespace

int dmrg_build_ops(dmrg_ctx* ctx, int prec) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(valid_prec(prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    x.build_ops(prec);
  });
}

int dmrg_sigma(dmrg_ctx* ctx, int site, int kind, int nvec, const double* C_in, double* sigma_out, size_t len,
               int prec) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    x.require_gpu();
    DMRG_REQUIRE(valid_prec(prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(kind >= DMRG_SIGMA_ZEROTH_1SITE && kind <= DMRG_SIGMA_TDA_DH_LEFT, DMRG_ERR_INVALID_ARG,
                 "unknown sigma kind");
    DMRG_REQUIRE(nvec >= 1 && C_in && sigma_out, DMRG_ERR_INVALID_ARG, "need nvec >= 1 and non-null arrays");
    DMRG_REQUIRE(x.have_mps, DMRG_ERR_STATE, "no MPS");
    const int width = kind == DMRG_SIGMA_ZEROTH_2SITE ? 2 : 1;
    DMRG_REQUIRE(site >= 0 && site + width <= x.L, DMRG_ERR_INVALID_ARG, "bad site");
    const size_t size = x.layout(site, width).size;
    DMRG_REQUIRE(len == size * size_t(nvec), DMRG_ERR_INVALID_ARG,
                 "len " + std::to_string(len) + " is not nvec * size = " + std::to_string(nvec) + " * " +
                     std::to_string(size));
    if (kind <= DMRG_SIGMA_ZEROTH_2SITE) x.sigma(site, width, nvec, C_in, sigma_out, prec);
    else x.sigma_tda(site, kind, nvec, C_in, sigma_out, prec);
  });
}

int dmrg_sigma_noalloc(dmrg_ctx* ctx, int site, int kind, int nvec, const double* C_in, double* sigma_out,
                       size_t len, int prec) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    x.require_gpu();
    DMRG_REQUIRE(valid_prec(prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(kind == DMRG_SIGMA_ZEROTH_1SITE || kind == DMRG_SIGMA_ZEROTH_2SITE, DMRG_ERR_INVALID_ARG,
                 "the no-allocation sigma takes the zeroth-order kinds only");
    DMRG_REQUIRE(nvec >= 1 && C_in && sigma_out, DMRG_ERR_INVALID_ARG, "need nvec >= 1 and non-null arrays");
    DMRG_REQUIRE(x.have_mps, DMRG_ERR_STATE, "no MPS");
    const int width = kind == DMRG_SIGMA_ZEROTH_2SITE ? 2 : 1;
    DMRG_REQUIRE(site >= 0 && site + width <= x.L, DMRG_ERR_INVALID_ARG, "bad site");
    const size_t size = x.layout(site, width).size;
    DMRG_REQUIRE(len == size * size_t(nvec), DMRG_ERR_INVALID_ARG, "len is not nvec * size");
    static_assert(DMRG_NOALLOC_SCRATCH_BYTES == (64u << 20), "scratch size of the header and the library");
    x.sigma_noalloc(site, width, nvec, C_in, sigma_out, prec);
  });
}

int dmrg_autotune(dmrg_ctx* ctx, int site, int nvec, int prec, int* shapes_out, double* best_ms_out) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(valid_prec(prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(shapes_out && best_ms_out, DMRG_ERR_INVALID_ARG, "null outputs");
    x.autotune(site, nvec, prec, shapes_out, best_ms_out);
  });
}

int dmrg_diag(dmrg_ctx* ctx, int site, int width, double* diag_out, size_t len, int prec) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    x.require_gpu();
    DMRG_REQUIRE(prec == DMRG_FP64, DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(diag_out, DMRG_ERR_INVALID_ARG, "null output");
    DMRG_REQUIRE(x.have_mps, DMRG_ERR_STATE, "no MPS");
    DMRG_REQUIRE(width >= 1 && width <= 2 && site >= 0 && site + width <= x.L, DMRG_ERR_INVALID_ARG,
                 "bad site/width");
    DMRG_REQUIRE(len == x.layout(site, width).size, DMRG_ERR_INVALID_ARG, "len is not the tensor size");
    x.diag(site, width, diag_out);
    x.sync();
  });
}

int dmrg_renormalize(dmrg_ctx* ctx, int site, int dir, int order, int nvec, const double* A1, size_t len,
                     int prec) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    x.require_gpu();
    DMRG_REQUIRE(order == DMRG_ZEROTH || order == DMRG_FIRST, DMRG_ERR_INVALID_ARG, "order must be 0 or 1");
    DMRG_REQUIRE(dir == DMRG_DIR_LEFT || dir == DMRG_DIR_RIGHT, DMRG_ERR_INVALID_ARG, "bad direction");
    DMRG_REQUIRE(valid_prec(prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(x.ops_prec >= 0, DMRG_ERR_STATE, "call dmrg_build_ops first");
    DMRG_REQUIRE(site >= 0 && site < x.L, DMRG_ERR_INVALID_ARG, "bad site");
    if (order == DMRG_FIRST) {
      DMRG_REQUIRE(nvec >= 1 && A1, DMRG_ERR_INVALID_ARG, "first order needs nvec >= 1 tensors");
      DMRG_REQUIRE(len == x.layout(site, 1).size * size_t(nvec), DMRG_ERR_INVALID_ARG,
                   "len is not nvec * size of the site tensor");
      x.renorm_first(site, dir, nvec, A1, prec);
      return;
    }
    DMRG_REQUIRE(nvec == 0 && !A1, DMRG_ERR_INVALID_ARG, "zeroth order takes no tensors (nvec 0, A1 NULL)");
    ++x.generation;
    if (dir == DMRG_DIR_LEFT) {
      x.renorm(DMRG_DIR_LEFT, site, x.site[site].L.as<double>(), x.site[site].L.as<double>(), 0, x.left[site],
               x.left[site + 1], false, 1, prec);
    } else {
      x.renorm(DMRG_DIR_RIGHT, site, x.site[site].R.as<double>(), x.site[site].R.as<double>(), 0,
               x.right[site + 1], x.right[site], false, 1, prec);
    }
    x.sync();
  });
}

int dmrg_sweep_ground(dmrg_ctx* ctx, const dmrg_sweep_params* p, double* energy, double* discarded) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(p && energy, DMRG_ERR_INVALID_ARG, "null arguments");
    DMRG_REQUIRE(valid_prec(p->prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    bool conv = true;
    x.sweep_ground(*p, energy, discarded, &conv);
  });
}

int dmrg_tda_roots(dmrg_ctx* ctx, int nroots, const dmrg_davidson_params* p, double* omega, double* e_total,
                   double* resid2, int* iters) {
  bool conv = false;
  int rc = guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(p, DMRG_ERR_INVALID_ARG, "null parameters");
    DMRG_REQUIRE(valid_prec(p->prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(p->polish == 0 || p->polish == -1, DMRG_ERR_INVALID_ARG, "polish must be 0 or -1");
    DMRG_REQUIRE(p->guess == 0 || p->guess == 1, DMRG_ERR_INVALID_ARG, "guess must be 0 or 1");
    x.tda_roots(nroots, *p, omega, e_total, resid2, iters, &conv);
  });
  if (rc == DMRG_OK && !conv) {
    ctx->x->err = "Davidson iteration limit reached";
    return DMRG_ERR_NOT_CONVERGED;
  }
  return rc;
}

int dmrg_tda_transition(dmrg_ctx* ctx, int nroots, const dmrg_davidson_params* p, double* omega, double* e_total,
                        double* resid2, int* iters, double* gamma) {
  bool conv = false;
  int rc = guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(p, DMRG_ERR_INVALID_ARG, "null parameters");
    DMRG_REQUIRE(valid_prec(p->prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(p->polish == 0 || p->polish == -1, DMRG_ERR_INVALID_ARG, "polish must be 0 or -1");
    DMRG_REQUIRE(p->guess == 0 || p->guess == 1, DMRG_ERR_INVALID_ARG, "guess must be 0 or 1");
    x.tda_transition(nroots, *p, omega, e_total, resid2, iters, &conv, gamma);
  });
  if (rc == DMRG_OK && !conv) {
    ctx->x->err = "Davidson iteration limit reached";
    return DMRG_ERR_NOT_CONVERGED;
  }
  return rc;
}

int dmrg_response(dmrg_ctx* ctx, const double* v, double omega, const dmrg_davidson_params* p, double* chi,
                  double* resid2, int* iters) {
  bool conv = false;
  int rc = guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(p, DMRG_ERR_INVALID_ARG, "null parameters");
    DMRG_REQUIRE(valid_prec(p->prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(p->polish == 0 || p->polish == -1, DMRG_ERR_INVALID_ARG, "polish must be 0 or -1");
    x.response(v, omega, *p, chi, resid2, iters, &conv);
  });
  if (rc == DMRG_OK && !conv) {
    ctx->x->err = "Davidson iteration limit reached";
    return DMRG_ERR_NOT_CONVERGED;
  }
  return rc;
}

int dmrg_rpa_roots(dmrg_ctx* ctx, int nroots, const dmrg_davidson_params* p, double* omega, double* e_total,
                   double* resid2, int* iters) {
  bool conv = false;
  int rc = guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(p, DMRG_ERR_INVALID_ARG, "null parameters");
    DMRG_REQUIRE(valid_prec(p->prec), DMRG_ERR_INVALID_ARG, "unsupported precision");
    DMRG_REQUIRE(p->polish == 0 || p->polish == -1, DMRG_ERR_INVALID_ARG, "polish must be 0 or -1");
    DMRG_REQUIRE(p->guess == 0 || p->guess == 1, DMRG_ERR_INVALID_ARG, "guess must be 0 or 1");
    x.rpa_roots(nroots, *p, omega, e_total, resid2, iters, &conv);
  });
  if (rc == DMRG_OK && !conv) {
    ctx->x->err = "Davidson iteration limit reached";
    return DMRG_ERR_NOT_CONVERGED;
  }
  return rc;
}

int dmrg_rpa_reduced(int l, const double* HR, const double* SR, const double* WR, double e0, int nroots,
                     double* omega_out, double* x_out, double* y_out) {
  if (l < 1 || l > 4096 || nroots < 1 || !HR || !SR || !WR || !omega_out) return DMRG_ERR_INVALID_ARG;
  try {
    dmrg::RpaReduced red;
    if (dmrg::rpa_reduced_solve(l, HR, SR, WR, e0, 1e-10, red) != 0) return DMRG_ERR_SINGULAR;
    if (red.r < nroots) return DMRG_ERR_SINGULAR;
    for (int k = 0; k < nroots; ++k) {
      omega_out[k] = red.omega[k];
      for (int u = 0; u < l; ++u) {
        double a = 0, b = 0;
        for (int t = 0; t < red.r; ++t) {
          a += red.T[u + size_t(t) * l] * red.x[t + size_t(k) * red.r];
          b += red.T[u + size_t(t) * l] * red.y[t + size_t(k) * red.r];
        }
        if (x_out) x_out[u + size_t(k) * l] = a;
        if (y_out) y_out[u + size_t(k) * l] = b;
      }
    }
    return red.r;
  } catch (...) {
    return DMRG_ERR_INTERNAL;
  }
}

int dmrg_tda_reduced(dmrg_ctx* ctx, int* l, double* HR, double* SR) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(l, DMRG_ERR_INVALID_ARG, "null l");
    DMRG_REQUIRE(x.tda_l > 0, DMRG_ERR_STATE, "no TDA run yet");
    *l = x.tda_l;
    if (HR) std::memcpy(HR, x.tda_hr.data(), x.tda_hr.size() * sizeof(double));
    if (SR) std::memcpy(SR, x.tda_sr.data(), x.tda_sr.size() * sizeof(double));
  });
}

int dmrg_get_stats(dmrg_ctx* ctx, dmrg_stats* out) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(out, DMRG_ERR_INVALID_ARG, "null stats");
    *out = x.stats;
  });
}

size_t dmrg_stats_size(void) { return sizeof(dmrg_stats); }

int dmrg_debug_mpo_dense(dmrg_ctx* ctx, int wide_bond, int from_right, double* out) {
  return guard(ctx, [&](dmrg::Ctx& x) {
    DMRG_REQUIRE(x.L <= 5 && out, DMRG_ERR_INVALID_ARG, "dense contraction only for L <= 5");
    DMRG_REQUIRE(wide_bond < x.L - 1, DMRG_ERR_INVALID_ARG, "bad wide bond");
    if (from_right) dmrg::debug_mpo_dense_right(*x.H, wide_bond, out);
    else dmrg::debug_mpo_dense_left(*x.H, wide_bond, out);
  });
}

}  // extern "C"
