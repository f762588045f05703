// Wave-equation functions c(t^2 A) = cos(t sqrt A) and s(t, A) = sin(t sqrt A) / sqrt A
// (Sections 1 and 2.2): the factorized schemes with B = t^2 A in the role of
// the paper's A_2 and the scalar t in the role of the final factor A, so each
// scheme spends one product fewer than its cos/sin parent and the sine's last
// "multiply by A" becomes a scalar folded into an epilogue.
//
// The norm/copy kernel writes Ap = B = t^2 A (zero padded) and plans on
// ||B||_1. With s double-angle steps the scheme runs on B_s = 4^-s B (the
// factor 4^-s goes into operand scales and epilogue coefficients, B_s is never
// formed) and t_s = 2^-s t. Launch sequences ("->" lists epilogue outputs):
//
// 2 products (P^c_4 of Algorithm4cA and P^s_{3,4}, with the B_4 term's sign
//   of Algorithm4sA):
//   G1 B2 = B_s B_s -> B2, W = -B_s/6! + B2/8!, Pc = I - B_s/2 + B2/24,
//                      Ps = t_s (I - B_s/6 + B2/120)
//   G2 B4 = B2 W    -> C = Pc + B4, S = Ps + (t_s/7) B4
// 3 products (P^c_4 and P^s_4): as above, G1 also writes
//   Ws = -B_s/7! + B2/9!, and
//   G2 B4 = B2 W    -> C = Pc + B4
//   G3 B4s = B2 Ws  -> S = Ps + t_s B4s
// 4 products (P^c_8 with eq:cosm8's coefficients, P^s_{8,12} with Algorithm6sA's):
//   G1 B2 = B_s B_s -> B2, W = x1 B_s + x2 B2
//   G2 B4 = B2 W    -> B4, L = x3 B2 + B4, R = x4 I + x5 B_s + x6 B2 + x7 B4,
//                      Pc = I - B_s/2 + x8 B2, Q = z5 (I + B_s) + z6 B2 + z7 B4,
//                      P = z0 I + z1 B_s + z2 B2 + z3 B4
//   G3 T = L R      -> C = Pc + T, Q += z8 C, P += z4 C
//   G4 U = Q B4     -> S = t_s (P + U)
// 5 products (P^c_12 with Coefs7cA, P^s_{11,24} with Coefs7sA):
//   G1 B2 = B_s B_s -> B2
//   G2 B3 = B2 B_s  -> D_j = a0j I + a1j B_s + a2j B2 + a3j B3 (j = 1..4),
//                      P = z0 I + z1 B_s + z2 B2 + z3 B3, Q = z6 I + z7 B_s + z8 B2 + z9 B3
//   G3 K = D4 D4    -> B6 = D3 + K, L = D2 + B6
//   G4 T = L B6     -> C = D1 + T, Q += z10 B6 + z11 C, P += z4 B6 + z5 C
//   G5 U = Q C      -> S = t_s (P + U)
// Double angle (Section 1), s times, from the old pair (C, S):
//   one launch, two problems sharing the right operand C:
//   [P | Q] = [C | S] C -> C' = 2 P - I, S' = 2 Q.
#include <math.h>
#include <string.h>

#include "schemes.hpp"
#include "coeffs.hpp"

namespace sc {

static sincosm_status wave2(Run& r, double bs, double ts, bool three) {
  const Modes& m = *r.m;
  const int64_t np = m.np;
  const int nv = (int)r.n;
  const bool pf = m.poly_f64;
  Problem p = make_problem(nv);
  add_seg(p, r.Ap, r.Ap, np, bs, bs);
  add_in(p, r.Ap, np);
  add_out(p, internal(r.W[1], m, pf), 1.0, 0.0, {});                                    // B2
  add_out(p, internal(r.W[2], m, pf), 1.0 / 40320.0, 0.0, {-bs / 720.0});               // W
  add_out(p, internal(r.W[3], m, pf), 1.0 / 24.0, 1.0, {-0.5 * bs});                    // Pc
  add_out(p, internal(r.W[4], m, pf), ts / 120.0, ts, {-ts * bs / 6.0});                // Ps
  if (three) add_out(p, internal(r.W[5], m, pf), 1.0 / 362880.0, 0.0, {-bs / 5040.0});  // Ws
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  p = make_problem(nv);
  add_seg(p, r.W[1], r.W[2], np);
  add_in(p, r.W[3], np);
  add_in(p, r.W[4], np);
  add_out(p, r.Cout, 1.0, 0.0, {1.0, 0.0});
  if (!three) {
    add_out(p, r.Sout, ts / 7.0, 0.0, {0.0, 1.0});
    return gemm(r, m.poly, one(p, (int)np));
  }
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  p = make_problem(nv);
  add_seg(p, r.W[1], r.W[5], np);
  add_in(p, r.W[4], np);
  add_out(p, r.Sout, ts, 0.0, {1.0});
  return gemm(r, m.poly, one(p, (int)np));
}

static sincosm_status wave4(Run& r, double bs, double ts) {
  const Modes& m = *r.m;
  const int64_t np = m.np;
  const int nv = (int)r.n;
  const bool pf = m.poly_f64;
  const Coeffs& k = coeffs();
  const double* x = k.x;
  const double* z = k.z6;
  Problem p = make_problem(nv);
  add_seg(p, r.Ap, r.Ap, np, bs, bs);
  add_in(p, r.Ap, np);
  add_out(p, internal(r.W[1], m, pf), 1.0, 0.0, {});             // B2
  add_out(p, internal(r.W[2], m, pf), x[2], 0.0, {x[1] * bs});   // W
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G2: B4 = B2 W; inputs B_s (Ap, scaled through the coefficients), B2 (W1)
  p = make_problem(nv);
  add_seg(p, r.W[1], r.W[2], np);
  add_in(p, r.Ap, np);
  add_in(p, r.W[1], np);
  add_out(p, internal(r.W[3], m, pf), 1.0, 0.0, {});                          // B4
  add_out(p, internal(r.W[4], m, pf), 1.0, 0.0, {0.0, x[3]});                 // L
  add_out(p, internal(r.W[5], m, pf), x[7], x[4], {x[5] * bs, x[6]});         // R
  add_out(p, internal(r.W[6], m, pf), 0.0, 1.0, {-0.5 * bs, x[8]});           // Pc
  add_out(p, internal(r.W[7], m, pf), z[7], z[5], {z[5] * bs, z[6]});         // Q
  add_out(p, internal(r.W[8], m, pf), z[3], z[0], {z[1] * bs, z[2]});         // P
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G3: T = L R; inputs Pc (W6), Q (W7), P (W8)
  p = make_problem(nv);
  add_seg(p, r.W[4], r.W[5], np);
  add_in(p, r.W[6], np);
  add_in(p, r.W[7], np);
  add_in(p, r.W[8], np);
  add_out(p, r.Cout, 1.0, 0.0, {1.0, 0.0, 0.0});                     // C = Pc + T
  add_out(p, internal(r.W[7], m, pf), z[8], 0.0, {z[8], 1.0, 0.0});  // Q + z8 C
  add_out(p, internal(r.W[8], m, pf), z[4], 0.0, {z[4], 0.0, 1.0});  // P + z4 C
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G4: U = Q B4 -> S = t_s (P + U)
  p = make_problem(nv);
  add_seg(p, r.W[7], r.W[3], np);
  add_in(p, r.W[8], np);
  add_out(p, r.Sout, ts, 0.0, {ts});
  return gemm(r, m.poly, one(p, (int)np));
}

static sincosm_status wave5(Run& r, double bs, double ts) {
  const Modes& m = *r.m;
  const int64_t np = m.np;
  const int nv = (int)r.n;
  const bool pf = m.poly_f64;
  const Coeffs& k = coeffs();
  const double(*a)[5] = k.a;
  const double* z = k.z7;
  Problem p = make_problem(nv);
  add_seg(p, r.Ap, r.Ap, np, bs, bs);
  add_out(p, internal(r.W[1], m, pf), 1.0, 0.0, {});   // B2
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G2: B3 = B2 B_s; inputs B_s (Ap), B2 (W1)
  p = make_problem(nv);
  add_seg(p, r.W[1], r.Ap, np, 1.0, bs);
  add_in(p, r.Ap, np);
  add_in(p, r.W[1], np);
  for (int j = 1; j <= 4; ++j)
    add_out(p, internal(r.W[1 + j], m, pf), a[3][j], a[0][j], {a[1][j] * bs, a[2][j]});  // D_j -> W2..W5
  add_out(p, internal(r.W[6], m, pf), z[3], z[0], {z[1] * bs, z[2]});                  // P
  add_out(p, internal(r.W[7], m, pf), z[9], z[6], {z[7] * bs, z[8]});                  // Q
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G3: K = D4 D4; inputs D3 (W4), D2 (W3) -> B6 = D3 + K (W4), L = D2 + B6 (W3)
  p = make_problem(nv);
  add_seg(p, r.W[5], r.W[5], np);
  add_in(p, r.W[4], np);
  add_in(p, r.W[3], np);
  add_out(p, internal(r.W[4], m, pf), 1.0, 0.0, {1.0, 0.0});
  add_out(p, internal(r.W[3], m, pf), 1.0, 0.0, {1.0, 1.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G4: T = L B6; inputs D1 (W2), B6 (W4), Q (W7), P (W6)
  p = make_problem(nv);
  add_seg(p, r.W[3], r.W[4], np);
  add_in(p, r.W[2], np);
  add_in(p, r.W[4], np);
  add_in(p, r.W[7], np);
  add_in(p, r.W[6], np);
  add_out(p, internal(r.W[8], m, pf), 1.0, 0.0, {1.0, 0.0, 0.0, 0.0});       // C (operand of G5)
  add_out(p, r.Cout, 1.0, 0.0, {1.0, 0.0, 0.0, 0.0});                        // C (result)
  add_out(p, internal(r.W[7], m, pf), z[11], 0.0, {z[11], z[10], 1.0, 0.0}); // Q + z10 B6 + z11 C
  add_out(p, internal(r.W[6], m, pf), z[5], 0.0, {z[5], z[4], 0.0, 1.0});    // P + z4 B6 + z5 C
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G5: U = Q C -> S = t_s (P + U)
  p = make_problem(nv);
  add_seg(p, r.W[7], r.W[8], np);
  add_in(p, r.W[6], np);
  add_out(p, r.Sout, ts, 0.0, {ts});
  return gemm(r, m.poly, one(p, (int)np));
}

static sincosm_status run_wave_scheme(Run& r, int level, double bs, double ts) {
  switch (level) {
    case 2: return wave2(r, bs, ts, false);
    case 3: return wave2(r, bs, ts, true);
    case 4: return wave4(r, bs, ts);
    default: return wave5(r, bs, ts);
  }
}

// One wave double-angle step: C' = 2 Cc Cc - I, S' = ks Sc Cc (ks = 2; 1 for
// S carried in units of t_s, see sincosm_wave_eval_async).
static sincosm_status wave_double_angle(Run& r, const void* Cc, const void* Sc, const Target& Cn,
                                        const Target& Sn, double ks = 2.0) {
  const Modes& m = *r.m;
  Problem p0 = make_problem((int)r.n);
  add_seg(p0, Cc, Cc, m.np);
  add_out(p0, Cn, 2.0, -1.0, {});
  Problem p1 = make_problem((int)r.n);
  add_seg(p1, Sc, Cc, m.np);
  add_out(p1, Sn, ks, 0.0, {});
  return gemm(r, m.sq, two(p0, p1, (int)m.np));
}

// State shared by the wave entry points after validation: modes, workspace
// layout, the padded B = t^2 A and the plan read back from the device.
struct WaveCall {
  Modes m;
  Layout L;
  char* base;
  hipStream_t stream;
  sincosm_plan plan;
};

// Validation common to every wave entry point (outputs are checked by the caller).
static sincosm_status wave_check(int64_t n, int dtype, const void* A, int64_t lda, double t, int acc, int prod,
                                 Modes& m) {
  if (n < 0 || n > (1 << 20)) return SINCOSM_E_ARG;
  if (acc != SINCOSM_ACC_DOUBLE && acc != SINCOSM_ACC_SINGLE) return SINCOSM_E_ARG;
  if (!isfinite(t)) return SINCOSM_E_ARG;
  if (!modes_for(n > 0 ? n : 1, dtype, prod, m)) return SINCOSM_E_ARG;
  if (n > 0 && (!A || lda < n)) return SINCOSM_E_ARG;
  if (m.poly == Arith::BF16X3 && !bf16x3_available()) return SINCOSM_E_UNSUPPORTED;
  return SINCOSM_OK;
}

// Workspace check, B = t^2 A padded copy, ||B||_1 and the wave plan.
static sincosm_status wave_prologue(int64_t n, const void* A, int64_t lda, double t, int acc, void* ws,
                                    size_t ws_bytes, void* stream, WaveCall& c) {
  c.L = layout_for(c.m);
  if (!ws || ws_bytes < c.L.total || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  c.stream = (hipStream_t)stream;
  c.base = (char*)ws;
  const NormScratch ns = norm_scratch(c.base + c.L.norm_off, c.m.np);
  SC_TRY(launch_norm_copy_plan(n, c.m.np, A, lda, c.m.user_f64, c.base + c.L.ap_off, c.m.poly_f64, acc, ns,
                               c.stream, 1, t * t));
  return read_plan(ns.plan, &c.plan, c.stream, 1, "wave", n);
}

// The wave scheme and the s double-angle steps. With user targets the last
// launch writes them; otherwise the final pair stays in the ping-pong
// buffers and *Cf, *Sf point at it.
static sincosm_status wave_body(WaveCall& c, int64_t n, double t, const Target* userC, const Target* userS,
                                const void** Cf, const void** Sf) {
  const Modes& m = c.m;
  Run r;
  r.m = &m;
  r.n = n;
  r.Ap = c.base + c.L.ap_off;
  for (int i = 0; i < 9; ++i) r.W[i] = c.base + c.L.w_off[i];
  r.i8ws = c.base + c.L.i8_off;
  r.stream = c.stream;
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = c.base + c.L.q_off[i];
  const int s = c.plan.s;
  const bool to_user = userC && userS;
  if (s == 0 && to_user) {
    r.Cout = *userC;
    r.Sout = *userS;
  } else {
    r.Cout = internal(Q[1], m, m.sq_f64);
    r.Sout = internal(Q[0], m, m.sq_f64);
  }
  const double bs = ldexp(1.0, -2 * s);
  const double ts = ldexp(t, -s);
  SC_TRY(run_wave_scheme(r, c.plan.level, bs, ts));
  const void* Cl = Q[1];
  const void* Sl = Q[0];
  for (int i = 0; i < s; ++i) {
    void* Sc = Q[(i & 1) ? 2 : 0];
    void* Cc = Q[(i & 1) ? 3 : 1];
    const bool last = (i == s - 1) && to_user;
    const Target Sn = last ? *userS : internal(Q[(i & 1) ? 0 : 2], m, m.sq_f64);
    const Target Cn = last ? *userC : internal(Q[(i & 1) ? 1 : 3], m, m.sq_f64);
    SC_TRY(wave_double_angle(r, Cc, Sc, Cn, Sn));
    Cl = Cn.p;
    Sl = Sn.p;
  }
  if (Cf) *Cf = Cl;
  if (Sf) *Sf = Sl;
  return SINCOSM_OK;
}

// Device-planned wave pair. The plan is decided on the device, so no scale
// that depends on s can reach a host-built epilogue coefficient; instead
//  - Ap is multiplied in place by 4^-s once the plan exists (B_s formed
//    explicitly: the same values the operand scales give), and
//  - the sine is carried in units of t_s: S~ = S / t_s. The scheme then
//    runs with t_s = 1, and since t_{j+1} = 2 t_j the step S' = 2 S C becomes
//    S~' = S~ C. The caller's S is t S~ after the last step.
// Schemes of levels 5, 4, 3, 2 packed into slot launches, s_max guarded
// steps; the pair ends in (Q1, Q0) for even s and (Q3, Q2) for odd s.
static sincosm_status wave_async_pair(WaveCall& c, int64_t n, const void* A, int64_t lda, double t, int acc,
                                      int s_max, sincosm_plan* plan_dev, const sincosm_plan** plan_rec) {
  const Modes& m = c.m;
  const NormScratch ns = norm_scratch(c.base + c.L.norm_off, m.np);
  void* Ap = c.base + c.L.ap_off;
  SC_TRY(launch_norm_copy_plan(n, m.np, A, lda, m.user_f64, Ap, m.poly_f64, acc, ns, c.stream, 1, t * t, s_max,
                               plan_dev));
  SC_TRY(launch_scale_by_plan(ns.plan, 2, Ap, m.np * m.np, m.poly_f64, c.stream));
  Run r;
  r.m = &m;
  r.n = n;
  r.Ap = Ap;
  for (int i = 0; i < 9; ++i) r.W[i] = c.base + c.L.w_off[i];
  r.i8ws = c.base + c.L.i8_off;
  r.stream = c.stream;
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = c.base + c.L.q_off[i];
  r.cond.plan = ns.plan;
  r.cond.level = 0;
  r.cond.step = -1;
  r.cond.select = 0;
  r.Cout = internal(Q[1], m, m.sq_f64);
  r.Sout = internal(Q[0], m, m.sq_f64);
  const int levels[4] = {5, 4, 3, 2};   // most products first
  SC_TRY(enqueue_by_slot(r, levels, 4, [](Run& rr, int level) { return run_wave_scheme(rr, level, 1.0, 1.0); }));
  for (int i = 0; i < s_max; ++i) {
    r.cond.step = i;
    void* Sc = Q[(i & 1) ? 2 : 0];
    void* Cc = Q[(i & 1) ? 3 : 1];
    const Target Sn = internal(Q[(i & 1) ? 0 : 2], m, m.sq_f64);
    const Target Cn = internal(Q[(i & 1) ? 1 : 3], m, m.sq_f64);
    SC_TRY(wave_double_angle(r, Cc, Sc, Cn, Sn, 1.0));
  }
  *plan_rec = ns.plan;
  return SINCOSM_OK;
}

}  // namespace sc

using namespace sc;

extern "C" {

sincosm_status sincosm_wave_plan_host(double normB, int acc, sincosm_plan* out) {
  if (!out || (acc != SINCOSM_ACC_DOUBLE && acc != SINCOSM_ACC_SINGLE)) return SINCOSM_E_ARG;
  plan_rule_wave(normB, acc, out);
  return SINCOSM_OK;
}

static void empty_plan(int acc, sincosm_plan* plan_host) {
  if (plan_host) { plan_rule_wave(0.0, acc, plan_host); plan_host->level = 0; plan_host->products = 0; }
}

sincosm_status sincosm_wave_eval(int64_t n, int dtype, const void* A, int64_t lda, double t, void* C,
                                 int64_t ldc, void* S, int64_t lds, int acc, int prod, void* ws,
                                 size_t ws_bytes, sincosm_plan* plan_host, void* stream) {
  WaveCall c;
  SC_TRY(wave_check(n, dtype, A, lda, t, acc, prod, c.m));
  if (n == 0) { empty_plan(acc, plan_host); return SINCOSM_OK; }
  if (!C || !S || ldc < n || lds < n) return SINCOSM_E_ARG;
  const size_t es = dtype == SINCOSM_F64 ? 8 : 4;
  if (overlaps(A, lda, C, ldc, n, es) || overlaps(A, lda, S, lds, n, es) || overlaps(C, ldc, S, lds, n, es))
    return SINCOSM_E_ARG;
  SC_TRY(wave_prologue(n, A, lda, t, acc, ws, ws_bytes, stream, c));
  if (plan_host) *plan_host = c.plan;
  if (c.plan.status != SINCOSM_OK) {
    SC_TRY(launch_fill_nan(n, C, ldc, c.m.user_f64, c.stream));
    SC_TRY(launch_fill_nan(n, S, lds, c.m.user_f64, c.stream));
    return SINCOSM_E_NONFINITE;
  }
  const Target userC{C, ldc, (int)n, c.m.user_f64};
  const Target userS{S, lds, (int)n, c.m.user_f64};
  return wave_body(c, n, t, &userC, &userS, nullptr, nullptr);
}

sincosm_status sincosm_wave_block_eval(int64_t n, int dtype, const void* A, int64_t lda, double t, void* E,
                                       int64_t lde, int acc, int prod, void* ws, size_t ws_bytes,
                                       sincosm_plan* plan_host, void* stream) {
  WaveCall c;
  SC_TRY(wave_check(n, dtype, A, lda, t, acc, prod, c.m));
  if (n == 0) { empty_plan(acc, plan_host); return SINCOSM_OK; }
  if (!E || lde < 2 * n) return SINCOSM_E_ARG;
  const size_t es = dtype == SINCOSM_F64 ? 8 : 4;
  {
    const char* a0 = (const char*)A;
    const char* a1 = a0 + ((size_t)(n - 1) * lda + n) * es;
    const char* e0 = (const char*)E;
    const char* e1 = e0 + ((size_t)(2 * n - 1) * lde + 2 * n) * es;
    if (a0 < e1 && e0 < a1) return SINCOSM_E_ARG;
  }
  SC_TRY(wave_prologue(n, A, lda, t, acc, ws, ws_bytes, stream, c));
  if (plan_host) *plan_host = c.plan;
  if (c.plan.status != SINCOSM_OK) {
    SC_TRY(launch_fill_nan_rect(2 * n, 2 * n, E, lde, c.m.user_f64, c.stream));
    return SINCOSM_E_NONFINITE;
  }
  const void* Cf = nullptr;
  const void* Sf = nullptr;
  SC_TRY(wave_body(c, n, t, nullptr, nullptr, &Cf, &Sf));
  // A (unscaled) padded into the ping-pong pair that does not hold the result
  const Modes& m = c.m;
  void* Q0 = c.base + c.L.q_off[0];
  void* Q2 = c.base + c.L.q_off[2];
  void* Ap = (Sf == Q0) ? Q2 : Q0;
  SC_TRY(launch_convert_pad(n, m.np, A, lda, m.user_f64, Ap, m.sq_f64, c.stream));
  // one launch: D = A s; E21 = -D, E11 = E22 = c, E12 = s
  char* e = (char*)E;
  const Target E11{e, lde, (int)n, m.user_f64};
  const Target E12{e + (size_t)n * es, lde, (int)n, m.user_f64};
  const Target E21{e + (size_t)n * lde * es, lde, (int)n, m.user_f64};
  const Target E22{e + ((size_t)n * lde + n) * es, lde, (int)n, m.user_f64};
  Problem p = make_problem((int)n);
  add_seg(p, Ap, Sf, m.np);
  add_in(p, Cf, m.np);
  add_in(p, Sf, m.np);
  add_out(p, E21, -1.0, 0.0, {});
  add_out(p, E11, 0.0, 0.0, {1.0, 0.0});
  add_out(p, E22, 0.0, 0.0, {1.0, 0.0});
  add_out(p, E12, 0.0, 0.0, {0.0, 1.0});
  const TimingMark tm = timing_begin(SINCOSM_TIMING_SCHEME, c.stream);
  const sincosm_status st = launch_gemm(m.sq, m.tile, one(p, (int)m.np), c.stream);
  timing_end(tm, c.stream);
  return st;
}

sincosm_status sincosm_wave_eval_async(int64_t n, int dtype, const void* A, int64_t lda, double t, void* C,
                                       int64_t ldc, void* S, int64_t lds, int acc, int prod, int32_t s_max,
                                       void* ws, size_t ws_bytes, sincosm_plan* plan_dev, void* stream) {
  if (s_max < 0 || s_max > 1100) return SINCOSM_E_ARG;
  WaveCall c;
  SC_TRY(wave_check(n, dtype, A, lda, t, acc, prod, c.m));
  if (n == 0) return SINCOSM_OK;
  if (!C || !S || ldc < n || lds < n) return SINCOSM_E_ARG;
  const size_t es = dtype == SINCOSM_F64 ? 8 : 4;
  if (overlaps(A, lda, C, ldc, n, es) || overlaps(A, lda, S, lds, n, es) || overlaps(C, ldc, S, lds, n, es))
    return SINCOSM_E_ARG;
  c.L = layout_for(c.m);
  if (!ws || ws_bytes < c.L.total || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  c.stream = (hipStream_t)stream;
  c.base = (char*)ws;
  const sincosm_plan* rec = nullptr;
  SC_TRY(wave_async_pair(c, n, A, lda, t, acc, s_max, plan_dev, &rec));
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = c.base + c.L.q_off[i];
  return launch_copy_result(rec, n, c.m.np, Q, C, ldc, S, lds, c.m.user_f64, c.stream, t);
}

sincosm_status sincosm_wave_block_eval_async(int64_t n, int dtype, const void* A, int64_t lda, double t, void* E,
                                             int64_t lde, int acc, int prod, int32_t s_max, void* ws,
                                             size_t ws_bytes, sincosm_plan* plan_dev, void* stream) {
  if (s_max < 0 || s_max > 1100) return SINCOSM_E_ARG;
  WaveCall c;
  SC_TRY(wave_check(n, dtype, A, lda, t, acc, prod, c.m));
  if (n == 0) return SINCOSM_OK;
  if (!E || lde < 2 * n) return SINCOSM_E_ARG;
  const size_t es = dtype == SINCOSM_F64 ? 8 : 4;
  {
    const char* a0 = (const char*)A;
    const char* a1 = a0 + ((size_t)(n - 1) * lda + n) * es;
    const char* e0 = (const char*)E;
    const char* e1 = e0 + ((size_t)(2 * n - 1) * lde + 2 * n) * es;
    if (a0 < e1 && e0 < a1) return SINCOSM_E_ARG;
  }
  c.L = layout_for(c.m);
  if (!ws || ws_bytes < c.L.total || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  c.stream = (hipStream_t)stream;
  c.base = (char*)ws;
  const sincosm_plan* rec = nullptr;
  SC_TRY(wave_async_pair(c, n, A, lda, t, acc, s_max, plan_dev, &rec));
  const Modes& m = c.m;
  void* Q[4];
  for (int i = 0; i < 4; ++i) Q[i] = c.base + c.L.q_off[i];
  // the pair (C, S~) into (Q1, Q0) whatever the parity of s, then A padded into Q2
  SC_TRY(launch_copy_pair_if_odd(rec, m.np, Q[3], Q[2], Q[1], Q[0], c.stream, m.sq_f64 ? 8 : 4));
  SC_TRY(launch_convert_pad(n, m.np, A, lda, m.user_f64, Q[2], m.sq_f64, c.stream));
  // one launch: D = A S~; E21 = -t D, E11 = E22 = C, E12 = t S~ (skipped when
  // the record's status is not SINCOSM_OK; E is then filled with NaN)
  char* e = (char*)E;
  const Target E11{e, lde, (int)n, m.user_f64};
  const Target E12{e + (size_t)n * es, lde, (int)n, m.user_f64};
  const Target E21{e + (size_t)n * lde * es, lde, (int)n, m.user_f64};
  const Target E22{e + ((size_t)n * lde + n) * es, lde, (int)n, m.user_f64};
  Problem p = make_problem((int)n);
  add_seg(p, Q[2], Q[0], m.np);
  add_in(p, Q[1], m.np);
  add_in(p, Q[0], m.np);
  add_out(p, E21, -t, 0.0, {});
  add_out(p, E11, 0.0, 0.0, {1.0, 0.0});
  add_out(p, E22, 0.0, 0.0, {1.0, 0.0});
  add_out(p, E12, 0.0, 0.0, {0.0, t});
  GemmLaunch g = one(p, (int)m.np);
  g.cond.plan = rec;
  g.cond.level = 0;
  g.cond.step = -1;
  g.cond.select = 0;
  SC_TRY(launch_gemm(m.sq, m.tile, g, c.stream));
  return launch_fill_nan_if_rect(rec, 2 * n, 2 * n, E, lde, m.user_f64, c.stream);
}

}  // extern "C"
