// Tonal optimisation (Section 4): the least-squares problem min ||B g - f||^2
// over the values g stored at the mask, with B = interpolation after the
// harmonic solve, solved by CG on the normal equations B^T B g = B^T f in the
// least-squares (CGLS) form. B^T B is never formed: each iteration applies B
// once (a solve with K_FF) and B^T once (transposed interpolation, then the
// same solve).
//
// The iteration is split into segments that each end with one solve, so the
// same code runs host-driven here (fi_tonal_opt) and batched in the server.
// Every scalar of the method (gamma = ||s||^2, ||q||^2, the step lengths) is
// computed and consumed on the device.
#include <cmath>

#include "internal.h"

namespace fi {

int Cgls::alloc() {
  if (M->d_tsc) return FI_OK;
  const int64_t m = M->m, P = M->P;
  int rc = 0;
  if ((rc = device_alloc(M, (void**)&M->d_tg, (size_t)std::max<int64_t>(m, 1) * 8)) ||
      (rc = device_alloc(M, (void**)&M->d_ts, (size_t)std::max<int64_t>(m, 1) * 8)) ||
      (rc = device_alloc(M, (void**)&M->d_tr, (size_t)P * 8)) ||
      (rc = device_alloc(M, (void**)&M->d_tq, (size_t)P * 8)) ||
      (rc = device_alloc(M, (void**)&M->d_ywarm, (size_t)std::max<int64_t>(M->n, 1) * 8)) ||
      (rc = device_alloc(M, (void**)&M->d_tsc, 8 * sizeof(double))))
    return rc;
  return FI_OK;
}

namespace {
double* gamma_slot(fi_mesh* M, int k) { return M->d_tsc + Cgls::kScGamma + (k & 1); }
}  // namespace

int Cgls::pre() {
  int rc = FI_OK;
  x0 = nullptr;
  switch (seg) {
    case kInpaint:  // B g0: g0 = f on the mask unless given
      if (!start_from_g && (rc = launch_gather_mask(M, f, g))) return rc;
      return launch_lift(M, g, M->d_b64);
    case kAdjoint:  // B^T r: t = R^T r, solve with t_F
      if ((rc = launch_raster_transpose(M, M->d_tr, M->d_tpart, wsqrt))) return rc;
      // t_F straight into the solve's right-hand side
      if ((rc = launch_gather_vertex(M, M->d_tpart, M->d_b64, M->d_tD))) return rc;
      if (warm) x0 = M->d_ywarm;
      return FI_OK;
    case kApplyP:  // q = B p
      return launch_lift(M, M->d_tg, M->d_b64);
    case kFinal:   // B g for the final error
      return launch_lift(M, g, M->d_b64);
    default:
      return fail(FI_E_INVALID, "CGLS: no solve in this segment");
  }
}

int Cgls::post() {
  int rc = FI_OK;
  double* p = M->d_tg;
  double* s = M->d_ts;
  double* r = M->d_tr;
  double* q = M->d_tq;
  double* sc = M->d_tsc;
  const int64_t m = M->m, P = M->P;
  switch (seg) {
    case kInpaint:  // r = f - B g0, ||r||^2
      if ((rc = launch_vertex_values(M, M->d_x64, g, M->d_uvert)) ||
          (rc = launch_raster(M, M->d_uvert, nullptr, nullptr, q, nullptr, nullptr, nullptr,
                              nullptr)) ||
          (rc = launch_pixel_residual(M, f, q, r, wsqrt)))
        return rc;
      return launch_dot(M, r, r, P, sc + kScRR0);
    case kAdjoint:  // s = t_D - K_DF y; first: p = s; later: p = s + (gamma_k / gamma_k-1) p
      if ((rc = launch_adjoint_tail(M, M->d_tD, M->d_x64, s))) return rc;
      if (use_warm && M->n > 0) {
        FI_HIP_TRY(hipMemcpyAsync(M->d_ywarm, M->d_x64, (size_t)M->n * sizeof(double),
                                  hipMemcpyDeviceToDevice, M->ctx->stream));
        warm = true;
      }
      if ((rc = launch_dot(M, s, s, m, gamma_slot(M, k)))) return rc;
      if (k == 0) {
        FI_HIP_TRY(hipMemcpyAsync(p, s, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice,
                                  M->ctx->stream));
        return FI_OK;
      }
      return launch_xpby_ratio(M, m, s, gamma_slot(M, k), gamma_slot(M, k - 1), p);
    case kApplyP: {  // alpha = gamma / ||q||^2; g += alpha p; r -= alpha q
      if ((rc = launch_vertex_values(M, M->d_x64, p, M->d_uvert))) return rc;
      if (wsqrt) {
        if ((rc = launch_raster(M, M->d_uvert, nullptr, nullptr, q, nullptr, nullptr, nullptr,
                                nullptr)) ||
            (rc = launch_scale(M, P, wsqrt, q)) || (rc = launch_dot(M, q, q, P, sc + kScQQ)))
          return rc;
      } else if ((rc = launch_interp_sq(M, M->d_uvert, q, sc + kScQQ))) {
        return rc;
      }
      if ((rc = launch_axpy2_ratio(M, m, P, gamma_slot(M, k), sc + kScQQ, p, g, q, r)))
        return rc;
      ++k;
      return FI_OK;
    }
    case kFinal:  // sum of squared errors of B g
      if ((rc = launch_vertex_values(M, M->d_x64, g, M->d_uvert)) ||
          (rc = launch_raster(M, M->d_uvert, nullptr, nullptr, q, nullptr, nullptr, nullptr,
                              nullptr)) ||
          (rc = launch_raster(M, nullptr, q, f, nullptr, nullptr, nullptr, nullptr, M->d_rpart)))
        return rc;
      return launch_reduce(M, M->d_rpart, raster_blocks(M), 1, sc + kScSSE);
    default:
      return fail(FI_E_INVALID, "CGLS: nothing to do after the last segment");
  }
}

namespace {

int read_scalars(fi_mesh* M, double* out, int count) {
  FI_HIP_TRY(hipMemcpyAsync(M->h_red, M->d_tsc, (size_t)count * sizeof(double),
                            hipMemcpyDeviceToHost, M->ctx->stream));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  for (int i = 0; i < count; ++i) out[i] = M->h_red[i];
  return FI_OK;
}

}  // namespace
}  // namespace fi

using namespace fi;

extern "C" int fi_tonal_opt(fi_mesh* M, const uint8_t* f_dev, double* g_dev,
                            const fi_tonal_opts* opts, fi_tonal_stats* stats) {
  if (!M || !M->ctx) return fail(FI_E_INVALID, "mesh is NULL");
  if (!f_dev || !g_dev) return fail(FI_E_INVALID, "f_dev and g_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  fi_tonal_opts o;
  fi_tonal_opts_default(&o);
  if (opts) {
    o = *opts;
    if (o.rtol < 0) o.rtol = 1e-8;
    if (o.max_outer <= 0) o.max_outer = 500;
  }
  const fi_solve_opts io = resolve_opts(opts ? &opts->inner : nullptr);
  fi_tonal_stats ts{};
  Cgls c;
  c.M = M;
  c.f = f_dev;
  c.g = g_dev;
  c.start_from_g = o.start_from_g != 0;
  c.use_warm = o.cold_adjoint == 0;
  int rc = c.alloc();
  if (rc) return rc;
  auto run = [&](Cgls::Seg seg) -> int {
    c.seg = seg;
    int r = c.pre();
    if (r) return r;
    fi_solve_stats st{};
    r = solve_free(M, &io, &st, c.x0);
    ts.inner_iterations += st.iterations;
    if (r) return r;
    if (st.status != FI_OK) return fail(FI_E_NO_CONVERGENCE, "inner solve did not converge");
    return c.post();
  };
  double sc[8] = {0};
  if ((rc = run(Cgls::kInpaint)) || (rc = run(Cgls::kAdjoint))) return rc;
  if ((rc = read_scalars(M, sc, 8))) return rc;
  const double s0 = std::sqrt(sc[Cgls::kScGamma]);
  if (!std::isfinite(s0)) return fail(FI_E_INVALID, "non-finite normal residual");
  ts.mse_initial = sc[Cgls::kScRR0] / (double)M->P;
  ts.rel_normal_residual = s0 > 0 ? 1.0 : 0.0;
  ts.status = FI_OK;
  int it = 0;
  if (s0 > 0) {
    ts.status = FI_E_NO_CONVERGENCE;
    // one host read per iteration: ||q||^2 and the new gamma together
    while (it < o.max_outer) {
      if ((rc = run(Cgls::kApplyP)) || (rc = run(Cgls::kAdjoint))) return rc;
      ++it;
      if ((rc = read_scalars(M, sc, 8))) return rc;
      ts.rel_normal_residual = std::sqrt(sc[Cgls::kScGamma + (c.k & 1)]) / s0;
      if (ts.rel_normal_residual <= o.rtol) {
        ts.status = FI_OK;
        break;
      }
      if (!(sc[Cgls::kScQQ] > 0)) break;  // B p = 0: the step had length 0, no progress
    }
  }
  ts.outer_iterations = it;
  if (o.rtol == 0.0) ts.status = FI_OK;  // a fixed number of iterations was asked for
  if ((rc = run(Cgls::kFinal))) return rc;
  if ((rc = read_scalars(M, sc, 8))) return rc;
  ts.mse_final = sc[Cgls::kScSSE] / (double)M->P;
  if (stats) *stats = ts;
  if (ts.status != FI_OK)
    return fail(FI_E_NO_CONVERGENCE, "tonal optimisation reached the outer iteration cap");
  return FI_OK;
}

extern "C" int fi_tonal_opt_rgb(fi_mesh* M, const uint8_t* f_dev, double* g_dev,
                                const fi_tonal_opts* opts, fi_tonal_stats* stats) {
  if (!M || !M->ctx) return fail(FI_E_INVALID, "mesh is NULL");
  if (!f_dev || !g_dev) return fail(FI_E_INVALID, "f_dev and g_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  fi_tonal_opts o;
  fi_tonal_opts_default(&o);
  if (opts) {
    o = *opts;
    if (o.rtol < 0) o.rtol = 1e-8;
    if (o.max_outer <= 0) o.max_outer = 500;
  }
  const fi_solve_opts io = resolve_opts(opts ? &opts->inner : nullptr);
  constexpr int C = kMaxRhs;
  fi_mesh* ch[C];
  int rc = channel_views(M, C, ch);
  if (rc) return rc;
  Cgls cg[C];
  fi_tonal_stats ts[C] = {};
  bool active[C];
  for (int c = 0; c < C; ++c) {
    cg[c].M = ch[c];
    cg[c].f = f_dev + (size_t)c * M->P;
    cg[c].g = g_dev + (size_t)c * M->m;
    cg[c].start_from_g = o.start_from_g != 0;
    cg[c].use_warm = o.cold_adjoint == 0;
    if ((rc = cg[c].alloc())) return rc;
    active[c] = true;
  }
  // One segment for the active channels: their right-hand sides, one
  // multi-right-hand-side solve, then each channel's own update.
  auto run = [&](Cgls::Seg seg) -> int {
    fi_mesh* act[C];
    const double* x0[C];
    int idx[C], na = 0;
    for (int c = 0; c < C; ++c) {
      if (!active[c]) continue;
      cg[c].seg = seg;
      int r = cg[c].pre();
      if (r) return r;
      act[na] = ch[c];
      x0[na] = cg[c].x0;
      idx[na++] = c;
    }
    if (na == 0) return FI_OK;
    fi_solve_stats st[C] = {};
    int r = solve_multi(act, na, &io, st, x0);
    for (int q = 0; q < na; ++q) ts[idx[q]].inner_iterations += st[q].iterations;
    if (r) return r;
    for (int q = 0; q < na; ++q)
      if (st[q].status != FI_OK) return fail(FI_E_NO_CONVERGENCE, "inner solve did not converge");
    for (int q = 0; q < na; ++q)
      if ((r = cg[idx[q]].post())) return r;
    return FI_OK;
  };
  double sc[8] = {0};
  double s0[C];
  if ((rc = run(Cgls::kInpaint)) || (rc = run(Cgls::kAdjoint))) return rc;
  for (int c = 0; c < C; ++c) {
    if ((rc = read_scalars(ch[c], sc, 8))) return rc;
    s0[c] = std::sqrt(sc[Cgls::kScGamma]);
    if (!std::isfinite(s0[c])) return fail(FI_E_INVALID, "non-finite normal residual");
    ts[c].mse_initial = sc[Cgls::kScRR0] / (double)M->P;
    ts[c].rel_normal_residual = s0[c] > 0 ? 1.0 : 0.0;
    ts[c].status = s0[c] > 0 ? FI_E_NO_CONVERGENCE : FI_OK;
    active[c] = s0[c] > 0;
  }
  for (int it = 0; it < o.max_outer; ++it) {
    bool any = false;
    for (int c = 0; c < C; ++c) any = any || active[c];
    if (!any) break;
    if ((rc = run(Cgls::kApplyP)) || (rc = run(Cgls::kAdjoint))) return rc;
    for (int c = 0; c < C; ++c) {
      if (!active[c]) continue;
      ++ts[c].outer_iterations;
      if ((rc = read_scalars(ch[c], sc, 8))) return rc;
      ts[c].rel_normal_residual = std::sqrt(sc[Cgls::kScGamma + (cg[c].k & 1)]) / s0[c];
      if (ts[c].rel_normal_residual <= o.rtol) {
        ts[c].status = FI_OK;
        active[c] = false;
      } else if (!(sc[Cgls::kScQQ] > 0)) {
        active[c] = false;  // B p = 0: no progress possible
      }
    }
  }
  for (int c = 0; c < C; ++c) {
    if (o.rtol == 0.0) ts[c].status = FI_OK;  // a fixed number of iterations was asked for
    active[c] = true;
  }
  if ((rc = run(Cgls::kFinal))) return rc;
  bool ok = true;
  for (int c = 0; c < C; ++c) {
    if ((rc = read_scalars(ch[c], sc, 8))) return rc;
    ts[c].mse_final = sc[Cgls::kScSSE] / (double)M->P;
    ok = ok && ts[c].status == FI_OK;
  }
  if (stats)
    for (int c = 0; c < C; ++c) stats[c] = ts[c];
  if (!ok) return fail(FI_E_NO_CONVERGENCE, "tonal optimisation of a channel reached the cap");
  return FI_OK;
}

extern "C" void fi_l1_opts_default(fi_l1_opts* o) {
  if (!o) return;
  fi_solve_opts_default(&o->inner);
  o->eps = 0.5;
  o->irls_iters = 8;
  o->cgls_iters = 20;
  o->start_from_g = 0;
}

extern "C" int fi_tonal_opt_l1(fi_mesh* M, const uint8_t* f_dev, double* g_dev,
                               const fi_l1_opts* opts, fi_l1_stats* stats, double* mae_hist) {
  if (!M || !M->ctx) return fail(FI_E_INVALID, "mesh is NULL");
  if (!f_dev || !g_dev) return fail(FI_E_INVALID, "f_dev and g_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  fi_l1_opts o;
  fi_l1_opts_default(&o);
  if (opts) {
    o = *opts;
    if (!(o.eps > 0)) return fail(FI_E_INVALID, "eps must be positive");
    if (o.irls_iters < 0 || o.cgls_iters < 0) return fail(FI_E_INVALID, "negative iteration count");
    o.inner = resolve_opts(&o.inner);
  }
  Cgls c;
  c.M = M;
  c.f = f_dev;
  c.g = g_dev;
  int rc = c.alloc();
  if (rc) return rc;
  if (!M->d_wsqrt && (rc = device_alloc(M, (void**)&M->d_wsqrt, (size_t)M->P * sizeof(double))))
    return rc;
  if (!o.start_from_g && (rc = launch_gather_mask(M, f_dev, g_dev))) return rc;
  fi_l1_stats st{};
  auto run = [&](Cgls::Seg seg) -> int {
    c.seg = seg;
    int r = c.pre();
    if (r) return r;
    fi_solve_stats ss{};
    r = solve_free(M, &o.inner, &ss, c.x0);
    st.inner_iterations += ss.iterations;
    if (r) return r;
    if (ss.status != FI_OK) return fail(FI_E_NO_CONVERGENCE, "inner solve did not converge");
    return c.post();
  };
  // B g and its errors (q = B g stays in the CGLS workspace for the weights)
  auto evaluate = [&](double* mae, double* mse) -> int {
    c.wsqrt = nullptr;
    int r = run(Cgls::kFinal);
    if (r) return r;
    if ((r = launch_abs_err(M, M->d_tq, f_dev, M->d_tsc + Cgls::kScAbs))) return r;
    double sc[8];
    if ((r = read_scalars(M, sc, 8))) return r;
    *mae = sc[Cgls::kScAbs] / (double)M->P;
    *mse = sc[Cgls::kScSSE] / (double)M->P;
    return FI_OK;
  };
  double mae = 0.0, mse = 0.0;
  if ((rc = evaluate(&mae, &mse))) return rc;
  st.mae_initial = mae;
  if (mae_hist) mae_hist[0] = mae;
  for (int k = 0; k < o.irls_iters; ++k) {
    if ((rc = launch_irls_weights(M, f_dev, M->d_tq, o.eps, M->d_wsqrt))) return rc;
    c.wsqrt = M->d_wsqrt;
    c.start_from_g = true;
    c.k = 0;
    if ((rc = run(Cgls::kInpaint)) || (rc = run(Cgls::kAdjoint))) return rc;
    for (int j = 0; j < o.cgls_iters; ++j)
      if ((rc = run(Cgls::kApplyP)) || (rc = run(Cgls::kAdjoint))) return rc;
    if ((rc = evaluate(&mae, &mse))) return rc;
    if (mae_hist) mae_hist[k + 1] = mae;
    ++st.irls_iters;
  }
  st.mae_final = mae;
  st.mse_final = mse;
  st.status = FI_OK;
  if (stats) *stats = st;
  return FI_OK;
}
