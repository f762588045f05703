// Unitary propagator U(t) = e^{-itA} = cos(tA) - i sin(tA) of a real matrix
// (eq:unitary, Section 1): the cos/sin method on X = tA with real products
// only, two per double-angle step, then one pass that interleaves the real
// part C and the imaginary part -S into the caller's complex matrix.
//
// The norm/copy kernel writes the padded copy of tA (each element multiplied
// by t in float64) and plans on ||tA||_1; the scheme and the double-angle
// steps are those of sincosm_eval, with every result kept in the ping-pong
// buffers until the final interleave.
#include <math.h>
#include <string.h>

#include "schemes.hpp"

using namespace sc;

extern "C" {

sincosm_status sincosm_expi_eval(int64_t n, int dtype, const void* A, int64_t lda, double t, void* U, int64_t ldu,
                                 int acc, int prod, void* ws, size_t ws_bytes, sincosm_plan* plan_host,
                                 void* stream_) {
  if (n < 0 || n > (1 << 20)) return SINCOSM_E_ARG;
  if (!acc_valid(acc, SINCOSM_PLAN_EXTENDED)) return SINCOSM_E_ARG;
  if (!isfinite(t)) return SINCOSM_E_ARG;
  Modes m;
  if (!modes_for(n > 0 ? n : 1, dtype, prod, m)) return SINCOSM_E_ARG;
  if (n == 0) {
    if (plan_host) { plan_rule(0.0, acc, plan_host); plan_host->level = 0; plan_host->products = 0; }
    return SINCOSM_OK;
  }
  if (!A || !U || lda < n || ldu < n) return SINCOSM_E_ARG;
  const size_t es = dtype == SINCOSM_F64 ? 8 : 4;
  {
    const char* a0 = (const char*)A;
    const char* a1 = a0 + ((size_t)(n - 1) * lda + n) * es;
    const char* u0 = (const char*)U;
    const char* u1 = u0 + ((size_t)(n - 1) * ldu + n) * 2 * es;
    if (a0 < u1 && u0 < a1) return SINCOSM_E_ARG;
  }
  if (((uintptr_t)U) & (2 * es - 1)) return SINCOSM_E_ARG;   // complex elements must be aligned pairs
  if (m.poly == Arith::BF16X3 && !bf16x3_available()) return SINCOSM_E_UNSUPPORTED;
  const Layout L = layout_for(m);
  if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  hipStream_t stream = (hipStream_t)stream_;
  char* base = (char*)ws;

  const NormScratch ns = norm_scratch(base + L.norm_off, m.np);
  void* Xp = base + L.ap_off;
  SC_TRY(launch_norm_copy_plan(n, m.np, A, lda, m.user_f64, Xp, m.poly_f64, acc, ns, stream, 0, t));
  sincosm_plan plan;
  SC_TRY(read_plan(ns.plan, &plan, stream, 1, "sincosm_expi_eval", n));
  if (plan_host) *plan_host = plan;
  if (plan.status != SINCOSM_OK) {
    SC_TRY(launch_fill_nan_rect(n, 2 * n, U, 2 * ldu, m.user_f64, stream));
    return SINCOSM_E_NONFINITE;
  }

  Run r;
  r.m = &m;
  r.n = n;
  r.Ap = Xp;
  for (int i = 0; i < 9; ++i) r.W[i] = base + L.w_off[i];
  r.i8ws = base + L.i8_off;
  r.stream = stream;
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = base + L.q_off[i];
  r.Cout = internal(Q[1], m, m.sq_f64);
  r.Sout = internal(Q[0], m, m.sq_f64);
  const int s = plan.s;
  SC_TRY(run_scheme(r, plan.level, ldexp(1.0, -s)));
  const void* Cf = Q[1];
  const void* Sf = Q[0];
  for (int i = 0; i < s; ++i) {
    void* Sc = Q[(i & 1) ? 2 : 0];
    void* Cc = Q[(i & 1) ? 3 : 1];
    const Target Sn = internal(Q[(i & 1) ? 0 : 2], m, m.sq_f64);
    const Target Cn = internal(Q[(i & 1) ? 1 : 3], m, m.sq_f64);
    SC_TRY(double_angle(r, Sc, Cc, Cn, Sn));
    Cf = Cn.p;
    Sf = Sn.p;
  }
  return launch_interleave(n, m.np, Cf, Sf, true, U, ldu, m.sq_f64, stream);
}

sincosm_status sincosm_expi_eval_async(int64_t n, int dtype, const void* A, int64_t lda, double t, void* U,
                                       int64_t ldu, int acc, int prod, int32_t s_max, void* ws, size_t ws_bytes,
                                       sincosm_plan* plan_dev, void* stream_) {
  if (n < 0 || n > (1 << 20) || s_max < 0 || s_max > 1100) return SINCOSM_E_ARG;
  if (!acc_valid(acc, SINCOSM_PLAN_EXTENDED)) return SINCOSM_E_ARG;
  if (!isfinite(t)) return SINCOSM_E_ARG;
  Modes m;
  if (!modes_for(n > 0 ? n : 1, dtype, prod, m)) return SINCOSM_E_ARG;
  if (n == 0) return SINCOSM_OK;
  if (!A || !U || lda < n || ldu < n) return SINCOSM_E_ARG;
  const size_t es = dtype == SINCOSM_F64 ? 8 : 4;
  {
    const char* a0 = (const char*)A;
    const char* a1 = a0 + ((size_t)(n - 1) * lda + n) * es;
    const char* u0 = (const char*)U;
    const char* u1 = u0 + ((size_t)(n - 1) * ldu + n) * 2 * es;
    if (a0 < u1 && u0 < a1) return SINCOSM_E_ARG;
  }
  if (((uintptr_t)U) & (2 * es - 1)) return SINCOSM_E_ARG;
  if (m.poly == Arith::BF16X3 && !bf16x3_available()) return SINCOSM_E_UNSUPPORTED;
  const Layout L = layout_for(m);
  if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  Run r;
  r.m = &m;
  r.n = n;
  r.stream = (hipStream_t)stream_;
  char* base = (char*)ws;
  const sincosm_plan* rec = nullptr;
  SC_TRY(enqueue_async_pair(r, L, base, A, lda, acc, t, s_max, plan_dev, &rec));
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = base + L.q_off[i];
  return launch_copy_result_complex(rec, n, m.np, Q, U, ldu, -1.0, m.user_f64, r.stream);
}

}  // extern "C"
