// C ABI of the forward path: validation, workspace layout, plan read-back,
// then the scheme's launch sequence (schemes.cpp) and the s double-angle steps.
// With the refined-norm flag the schemes' first product A^2 is formed before
// the plan (its 1-norm refines theta) and reused after scaling by 4^-s.
#include <math.h>
#include <string.h>

#include "schemes.hpp"

using namespace sc;

namespace {

// The launches that follow the plan: the scheme on 2^-s A (its products read
// the padded copy in the workspace) and the s double-angle steps, ping-pong
// between (Q0, Q1) and (Q2, Q3); the last step (or the scheme when s = 0)
// writes the caller's C and S.
sincosm_status enqueue_method(Run& r, const Modes& m, const Layout& L, char* base, const sincosm_plan& plan,
                              const Target& userC, const Target& userS) {
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = base + L.q_off[i];
  const int s = plan.s;
  if (s == 0) {
    r.Cout = userC;
    r.Sout = userS;
  } else {
    r.Cout = internal(Q[1], m, m.sq_f64);
    r.Sout = internal(Q[0], m, m.sq_f64);
  }
  const double sx = ldexp(1.0, -s);
  SC_TRY(run_scheme(r, plan.level, sx));
  for (int i = 0; i < s; ++i) {
    void* Sc = Q[(i & 1) ? 2 : 0];
    void* Cc = Q[(i & 1) ? 3 : 1];
    const bool last = (i == s - 1);
    const Target Sn = last ? userS : internal(Q[(i & 1) ? 0 : 2], m, m.sq_f64);
    const Target Cn = last ? userC : internal(Q[(i & 1) ? 1 : 3], m, m.sq_f64);
    SC_TRY(double_angle(r, Sc, Cc, Cn, Sn));
  }
  return SINCOSM_OK;
}

}  // namespace

namespace sc {

// Launch sequences of several schemes, for a plan decided on the device: each
// level's sequence is recorded (fn(r, level)), then the sequences are packed
// into "slot" launches of up to MAX_PROB alternative problems (one per level,
// each level's products in increasing slots; levels listed first are placed
// first, each in the earliest slots with room), and every slot is launched
// with select = 1, so the device computes the problem of the plan's level.
sincosm_status enqueue_by_slot(Run& r, const int* levels, int nlev, SchemeFn fn) {
  constexpr int MAX_LEVELS = 8;
  constexpr int MAX_SLOTS = 12;
  if (nlev < 1 || nlev > MAX_LEVELS) return SINCOSM_E_ARG;
  Recorder rec[MAX_LEVELS];
  GemmLaunch slot[MAX_SLOTS];
  int fill[MAX_SLOTS] = {0};
  int nslots = 0;
  for (int li = 0; li < nlev; ++li) {
    Run rr = r;
    rr.rec = &rec[li];
    SC_TRY(fn(rr, levels[li]));
    int next = 0;
    for (int k = 0; k < rec[li].count; ++k) {
      const GemmLaunch& g = rec[li].launches[k];
      if (g.nprob != 1) return SINCOSM_E_ARG;   // scheme products are single problems
      while (next < nslots && fill[next] >= MAX_PROB) ++next;
      if (next == nslots) {
        if (nslots == MAX_SLOTS) return SINCOSM_E_ARG;
        memset(&slot[nslots], 0, sizeof(GemmLaunch));
        slot[nslots].np = g.np;
        ++nslots;
      }
      GemmLaunch& sl = slot[next];
      sl.prob[fill[next]] = g.prob[0];
      sl.cond.prob_level[fill[next]] = levels[li];
      ++fill[next];
      sl.nprob = fill[next];
      ++next;
    }
  }
  for (int k = 0; k < nslots; ++k) {
    DevCond c = r.cond;
    c.level = 0;
    c.step = -1;
    c.select = 1;
    for (int q = 0; q < MAX_PROB; ++q) c.prob_level[q] = q < fill[k] ? slot[k].cond.prob_level[q] : 0;
    Run rr = r;
    rr.cond = c;
    SC_TRY(gemm(rr, r.m->poly, slot[k]));
  }
  return SINCOSM_OK;
}

// The cos/sin schemes' products after the shared first one (r.y_ready set):
// without the extended flag, 6 launches for the 16 products of levels 7, 6, 4
// and 3.
sincosm_status enqueue_schemes_by_slot(Run& r, int acc) {
  const bool extended = (acc & SINCOSM_PLAN_EXTENDED) != 0;
  const int all[5] = {7, 6, 5, 4, 3};   // most products first
  const int base[4] = {7, 6, 4, 3};
  return enqueue_by_slot(r, extended ? all : base, extended ? 5 : 4,
                         [](Run& rr, int level) { return run_scheme(rr, level, SCALE_2_POW_MINUS_S); });
}

sincosm_status enqueue_async_pair(Run& r, const Layout& L, char* base, const void* A, int64_t lda, int acc,
                                  double pre, int s_max, sincosm_plan* plan_dev, const sincosm_plan** plan_rec) {
  const Modes& m = *r.m;
  const NormScratch ns = norm_scratch(base + L.norm_off, m.np);
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = base + L.q_off[i];
  r.Ap = base + L.ap_off;
  for (int i = 0; i < 9; ++i) r.W[i] = base + L.w_off[i];
  r.i8ws = base + L.i8_off;
  SC_TRY(launch_norm_copy_plan(r.n, m.np, A, lda, m.user_f64, base + L.ap_off, m.poly_f64, acc, ns, r.stream, 0,
                               pre, s_max, plan_dev));
  // Every product launch below reads the plan record. The scheme writes (C, S)
  // to (Q1, Q0) and the double-angle steps ping-pong between (Q1, Q0) and
  // (Q3, Q2); the caller then takes the pair that the record's s selects.
  r.cond.plan = ns.plan;
  r.cond.level = 0;
  r.cond.step = -1;
  r.cond.select = 0;
  r.Cout = internal(Q[1], m, m.sq_f64);
  r.Sout = internal(Q[0], m, m.sq_f64);
  SC_TRY(first_product(r, SCALE_2_POW_MINUS_S));   // shared by every scheme
  r.y_ready = true;
  SC_TRY(enqueue_schemes_by_slot(r, acc));
  r.cond.level = 0;
  for (int i = 0; i < s_max; ++i) {
    r.cond.step = i;
    void* Sc = Q[(i & 1) ? 2 : 0];
    void* Cc = Q[(i & 1) ? 3 : 1];
    const Target Sn = internal(Q[(i & 1) ? 0 : 2], m, m.sq_f64);
    const Target Cn = internal(Q[(i & 1) ? 1 : 3], m, m.sq_f64);
    SC_TRY(double_angle(r, Sc, Cc, Cn, Sn));
  }
  *plan_rec = ns.plan;
  return SINCOSM_OK;
}

}  // namespace sc

namespace {

// Argument and workspace checks shared by sincosm_eval and sincosm_eval_planned
// (n > 0, Modes already derived).
sincosm_status check_eval_args(int64_t n, int dtype, const void* A, int64_t lda, const void* C, int64_t ldc,
                               const void* S, int64_t lds, const Modes& m, void* ws, size_t ws_bytes) {
  if (!A || !C || !S) return SINCOSM_E_ARG;
  if (lda < n || ldc < n || lds < n) return SINCOSM_E_ARG;
  const size_t es = dtype == SINCOSM_F64 ? 8 : 4;
  if (overlaps(A, lda, C, ldc, n, es) || overlaps(A, lda, S, lds, n, es) || overlaps(C, ldc, S, lds, n, es))
    return SINCOSM_E_ARG;
  if (m.poly == Arith::BF16X3 && !bf16x3_available()) return SINCOSM_E_UNSUPPORTED;
  const Layout L = layout_for(m);
  if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  return SINCOSM_OK;
}

}  // namespace

namespace sc {

sincosm_status eval_planned(int64_t n, int dtype, const void* A, int64_t lda, void* C, int64_t ldc, void* S,
                            int64_t lds, int acc, int prod, const sincosm_plan* plan_in, void* ws,
                            size_t ws_bytes, sincosm_plan* plan_dev, hipStream_t stream, bool timed) {
  if (n < 0 || n > (1 << 20) || !plan_in) return SINCOSM_E_ARG;
  if (!acc_valid(acc, SINCOSM_PLAN_EXTENDED)) return SINCOSM_E_ARG;
  const int level = plan_in->level, s = plan_in->s;
  const bool level_ok = level == 3 || level == 4 || level == 6 || level == 7 ||
                        (level == 5 && (acc & SINCOSM_PLAN_EXTENDED));
  if (!level_ok || s < 0 || s > 1100) return SINCOSM_E_ARG;
  Modes m;
  if (!modes_for(n > 0 ? n : 1, dtype, prod, m)) return SINCOSM_E_ARG;
  if (n == 0) return SINCOSM_OK;
  SC_TRY(check_eval_args(n, dtype, A, lda, C, ldc, S, lds, m, ws, ws_bytes));
  const Layout L = layout_for(m);
  char* base = (char*)ws;
  const NormScratch ns = norm_scratch(base + L.norm_off, m.np);
  void* Ap = base + L.ap_off;
  Run r;
  r.m = &m;
  r.n = n;
  r.Ap = Ap;
  for (int i = 0; i < 9; ++i) r.W[i] = base + L.w_off[i];
  r.i8ws = base + L.i8_off;
  r.stream = stream;
  r.timed = timed;
  SC_TRY(launch_norm_copy_plan(n, m.np, A, lda, m.user_f64, Ap, m.poly_f64, acc, ns, stream));
  SC_TRY(launch_check_plan(acc, level, s, ns, plan_dev, stream));
  sincosm_plan plan;
  plan.level = level;
  plan.s = s;
  plan.products = level + 2 * s;
  plan.status = SINCOSM_OK;
  plan.norm1 = 0.0;
  const Target userC{C, ldc, (int)n, m.user_f64};
  const Target userS{S, lds, (int)n, m.user_f64};
  SC_TRY(enqueue_method(r, m, L, base, plan, userC, userS));
  SC_TRY(launch_fill_nan_if(ns.plan, n, C, ldc, m.user_f64, stream));
  return launch_fill_nan_if(ns.plan, n, S, lds, m.user_f64, stream);
}

}  // namespace sc

extern "C" {

const char* sincosm_strerror(int status) {
  switch (status) {
    case SINCOSM_OK: return "ok";
    case SINCOSM_E_ARG: return "invalid argument";
    case SINCOSM_E_UNSUPPORTED: return "unsupported combination";
    case SINCOSM_E_WORKSPACE: return "workspace missing or too small";
    case SINCOSM_E_NONFINITE: return "input holds Inf or NaN";
    case SINCOSM_E_HIP: return "HIP runtime error";
    case SINCOSM_E_PLAN: return "the given plan does not cover the matrix 1-norm";
    case SINCOSM_E_TOO_LARGE: return "the matrix needs more workspace than the static scratch holds";
    case SINCOSM_E_SCALING: return "the plan needs more double-angle steps than the call allowed";
    default: return "unknown status";
  }
}

sincosm_status sincosm_plan_host(double norm1, int acc, sincosm_plan* out) {
  if (!out || (!acc_valid(acc, SINCOSM_PLAN_EXTENDED))) return SINCOSM_E_ARG;
  plan_rule(norm1, acc, out);
  return SINCOSM_OK;
}

size_t sincosm_plan_workspace_size(int64_t n) {
  if (n <= 0) return 0;
  return align_up(norm_scratch_bytes(n), 256);
}

sincosm_status sincosm_plan_device(int64_t n, int dtype, const void* A, int64_t lda, int acc, void* ws,
                                   size_t ws_bytes, sincosm_plan* plan_host, void* stream_) {
  if (n < 0 || !plan_host) return SINCOSM_E_ARG;
  if (!acc_valid(acc, SINCOSM_PLAN_EXTENDED)) return SINCOSM_E_ARG;
  if (dtype != SINCOSM_F64 && dtype != SINCOSM_F32) return SINCOSM_E_ARG;
  if (n == 0) { plan_rule(0.0, acc, plan_host); return SINCOSM_OK; }
  if (!A || lda < n) return SINCOSM_E_ARG;
  if (!ws || ws_bytes < sincosm_plan_workspace_size(n) || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  hipStream_t stream = (hipStream_t)stream_;
  const NormScratch ns = norm_scratch(ws, n);
  SC_TRY(launch_norm_copy_plan(n, n, A, lda, dtype == SINCOSM_F64, nullptr, true, acc, ns, stream));
  return read_plan(ns.plan, plan_host, stream, 1, "sincosm_plan_device", n);
}

size_t sincosm_workspace_size(int64_t n, int dtype, int acc, int prod) {
  (void)acc;
  if (n <= 0) return 0;
  Modes m;
  if (!modes_for(n, dtype, prod, m)) return 0;
  return layout_for(m).total;
}

sincosm_status sincosm_eval(int64_t n, int dtype, const void* A, int64_t lda, void* C, int64_t ldc, void* S,
                            int64_t lds, int acc, int prod, void* ws, size_t ws_bytes, sincosm_plan* plan_host,
                            void* stream_) {
  if (n < 0 || n > (1 << 20)) return SINCOSM_E_ARG;
  if (!acc_valid(acc, SINCOSM_PLAN_EXTENDED | SINCOSM_PLAN_REFINED)) return SINCOSM_E_ARG;
  const bool refined = (acc & SINCOSM_PLAN_REFINED) != 0;
  acc &= ~(int)SINCOSM_PLAN_REFINED;
  Modes m;
  if (!modes_for(n > 0 ? n : 1, dtype, prod, m)) return SINCOSM_E_ARG;
  if (n == 0) {
    if (plan_host) { plan_rule(0.0, acc, plan_host); plan_host->level = 0; plan_host->products = 0; }
    return SINCOSM_OK;
  }
  SC_TRY(check_eval_args(n, dtype, A, lda, C, ldc, S, lds, m, ws, ws_bytes));
  const Layout L = layout_for(m);
  hipStream_t stream = (hipStream_t)stream_;
  char* base = (char*)ws;

  const NormScratch ns = norm_scratch(base + L.norm_off, m.np);
  void* Ap = base + L.ap_off;
  Run r;
  r.m = &m;
  r.n = n;
  r.Ap = Ap;
  for (int i = 0; i < 9; ++i) r.W[i] = base + L.w_off[i];
  r.i8ws = base + L.i8_off;
  r.stream = stream;
  SC_TRY(launch_norm_copy_plan(n, m.np, A, lda, m.user_f64, Ap, m.poly_f64, acc, ns, stream));
  sincosm_plan plans[2];
  if (refined) {
    // the schemes' first product, unscaled: W0 = A A; plan on min(||A||_1, ||A^2||_1^(1/2))
    Problem p = make_problem((int)n);
    add_seg(p, Ap, Ap, m.np);
    add_out(p, internal(r.W[0], m, m.poly_f64), 1.0, 0.0, {});
    SC_TRY(gemm(r, m.poly, one(p, (int)m.np)));
    SC_TRY(launch_norm_sq_plan(n, m.np, r.W[0], m.poly_f64, acc, ns, stream));
    SC_TRY(read_plan(ns.plan, plans, stream, 2, "sincosm_eval", n));
  } else {
    SC_TRY(read_plan(ns.plan, plans, stream, 1, "sincosm_eval", n));
  }
  const sincosm_plan plan = plans[0];
  if (plan_host) *plan_host = plan;
  if (plan.status != SINCOSM_OK) {
    SC_TRY(launch_fill_nan(n, C, ldc, m.user_f64, stream));
    SC_TRY(launch_fill_nan(n, S, lds, m.user_f64, stream));
    return SINCOSM_E_NONFINITE;
  }
  if (refined && plans[1].level == 1) {
    // reuse A^2 as Y = 4^-s A^2 (exact scaling, in place, epilogue-only launch)
    if (plan.s > 0) {
      Problem p = make_problem((int)n);
      add_in(p, r.W[0], m.np);
      add_out(p, internal(r.W[0], m, m.poly_f64), 0.0, 0.0, {ldexp(1.0, -2 * plan.s)});
      SC_TRY(launch_gemm(m.poly, m.tile, one(p, (int)m.np), stream));
    }
    r.y_ready = true;
  }
  const Target userC{C, ldc, (int)n, m.user_f64};
  const Target userS{S, lds, (int)n, m.user_f64};
  return enqueue_method(r, m, L, base, plan, userC, userS);
}

sincosm_status sincosm_eval_planned(int64_t n, int dtype, const void* A, int64_t lda, void* C, int64_t ldc,
                                    void* S, int64_t lds, int acc, int prod, const sincosm_plan* plan_in,
                                    void* ws, size_t ws_bytes, sincosm_plan* plan_dev, void* stream_) {
  return eval_planned(n, dtype, A, lda, C, ldc, S, lds, acc, prod, plan_in, ws, ws_bytes, plan_dev,
                      (hipStream_t)stream_, true);
}

sincosm_status sincosm_eval_async(int64_t n, int dtype, const void* A, int64_t lda, void* C, int64_t ldc, void* S,
                                  int64_t lds, int acc, int prod, int32_t s_max, void* ws, size_t ws_bytes,
                                  sincosm_plan* plan_dev, void* stream_) {
  if (n < 0 || n > (1 << 20) || s_max < 0 || s_max > 1100) return SINCOSM_E_ARG;
  if (!acc_valid(acc, SINCOSM_PLAN_EXTENDED)) return SINCOSM_E_ARG;
  Modes m;
  if (!modes_for(n > 0 ? n : 1, dtype, prod, m)) return SINCOSM_E_ARG;
  if (n == 0) return SINCOSM_OK;
  SC_TRY(check_eval_args(n, dtype, A, lda, C, ldc, S, lds, m, ws, ws_bytes));
  const Layout L = layout_for(m);
  Run r;
  r.m = &m;
  r.n = n;
  r.stream = (hipStream_t)stream_;
  char* base = (char*)ws;
  const sincosm_plan* rec = nullptr;
  SC_TRY(enqueue_async_pair(r, L, base, A, lda, acc, 1.0, s_max, plan_dev, &rec));
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = base + L.q_off[i];
  return launch_copy_result(rec, n, m.np, Q, C, ldc, S, lds, m.user_f64, r.stream);
}

size_t sincosm_matmul_workspace_size(int64_t n, int dtype, int prod) {
  if (n <= 0) return 0;
  Modes m;
  if (!modes_for(n, dtype, prod, m)) return 0;
  const size_t pe = m.poly_f64 ? 8 : 4;
  return 2 * align_up((size_t)m.np * m.np * pe, 256) +
         (m.poly == Arith::I8X5 ? align_up(i8x5_scratch_bytes(m.np), 256) : 0);
}

sincosm_status sincosm_matmul(int64_t n, int dtype, const void* X, int64_t ldx, const void* Y, int64_t ldy,
                              void* Z, int64_t ldz, int prod, void* ws, size_t ws_bytes, void* stream_) {
  if (n < 0) return SINCOSM_E_ARG;
  if (n == 0) return SINCOSM_OK;
  Modes m;
  if (!modes_for(n, dtype, prod, m)) return SINCOSM_E_ARG;
  if (!X || !Y || !Z || ldx < n || ldy < n || ldz < n) return SINCOSM_E_ARG;
  if (m.poly == Arith::BF16X3 && !bf16x3_available()) return SINCOSM_E_UNSUPPORTED;
  const size_t need = sincosm_matmul_workspace_size(n, dtype, prod);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  hipStream_t stream = (hipStream_t)stream_;
  char* base = (char*)ws;
  const size_t mat = align_up((size_t)m.np * m.np * (m.poly_f64 ? 8 : 4), 256);
  void* Xp = base;
  void* Yp = base + mat;
  SC_TRY(launch_convert_pad(n, m.np, X, ldx, m.user_f64, Xp, m.poly_f64, stream));
  SC_TRY(launch_convert_pad(n, m.np, Y, ldy, m.user_f64, Yp, m.poly_f64, stream));
  Problem p = make_problem((int)n);
  add_seg(p, Xp, Yp, m.np);
  add_out(p, Target{Z, ldz, (int)n, m.user_f64}, 1.0, 0.0, {});
  return launch_gemm(m.poly, m.tile, one(p, (int)m.np), stream, base + 2 * mat);
}

}  // extern "C"
