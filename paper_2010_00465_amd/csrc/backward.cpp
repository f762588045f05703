// Reverse pass: gradient of L(A) = <Gc, cos A> + <Gs, sin A> through the same
// computation the forward performs (same plan, same scheme, same steps).
//
// Every intermediate M of the forward is a polynomial in A, so M(A^T) = M(A)^T.
// The reverse pass therefore first runs the forward on B = A^T, keeping the
// scheme's intermediates and the inputs (S_i, C_i) of the double-angle steps;
// then each adjoint product of a forward product Z = X Y,
//   Xbar += Zbar Y^T = Zbar Y(B),   Ybar += X^T Zbar = X(B) Zbar,
// is a plain product of stored matrices, and the adjoints of the fused linear
// combinations are themselves linear combinations, fused into the epilogues
// of the adjoint products. Products that share an output are summed in one
// launch by giving it several k-segments.
//
// Double-angle step C' = I - 2 S S, S' = 2 S C (Section 1), adjoint:
//   Sbar = -2 C'bar S^T - 2 S^T C'bar + 2 S'bar C^T
//   Cbar =  2 S^T S'bar
// as one launch of three problems with 2, 1 and 1 k-segments (the first two
// terms of Sbar; Cbar; the last term of Sbar into a scratch matrix), so that
// no tile carries more than twice the work of another, then an epilogue-only
// launch adds the scratch matrix into Sbar.
// The scaled argument X = 2^-s A enters the first and last scheme products:
//   Abar = 2^-s Sbar0 V^T + 4^-s (Ybar A^T + A^T Ybar)    (one launch, 3 segments)
// Forward product count Pi + 2s; reverse 2 Pi + 4s, plus the recomputed
// forward on B (Pi + 2(s - 1)).
#include <math.h>
#include <string.h>

#include "coeffs.hpp"
#include "schemes.hpp"

namespace sc {
namespace {

struct BwdLayout {
  size_t norm_off, bp_off, w_off[9], rev_off[9], cot_off[4], chain_off, total;
  int s;
};

BwdLayout bwd_layout(const Modes& m, int s) {
  BwdLayout L;
  const size_t mat = align_up((size_t)m.np * m.np * 8, 256);
  size_t off = 0;
  L.norm_off = off; off += align_up(norm_scratch_bytes(m.np), 256);
  L.bp_off = off; off += mat;
  for (int i = 0; i < 9; ++i) { L.w_off[i] = off; off += mat; }
  for (int i = 0; i < 9; ++i) { L.rev_off[i] = off; off += mat; }
  for (int i = 0; i < 4; ++i) { L.cot_off[i] = off; off += mat; }
  L.chain_off = off; off += mat * (size_t)(2 * (s > 0 ? s : 0));
  L.total = off;
  L.s = s;
  return L;
}

struct Rev {
  Run* r;
  const Modes* m;
  const void* Bp;
  void* const* W;   // forward intermediates on B
  void* R[9];       // adjoint buffers
  const void* Cbar; // adjoint of the scheme's cosine output
  const void* Sbar; // adjoint of the scheme's sine output
  Target gA;
  double sx;
};

Target T(void* p, const Modes& m) { return internal(p, m, true); }

sincosm_status G(Rev& v, const GemmLaunch& g) { return gemm(*v.r, Arith::F64, g, SINCOSM_TIMING_BACKWARD); }

// Abar = sx Sbar V^T + (sx Ybar)(sx A^T) + (sx A^T)(sx Ybar)
sincosm_status final_abar(Rev& v, const void* VB, const void* Ybar) {
  const int64_t np = v.m->np;
  Problem p = make_problem((int)v.r->n);
  add_seg(p, v.Sbar, VB, np, v.sx, 1.0);
  add_seg(p, Ybar, v.Bp, np, v.sx, v.sx);
  add_seg(p, v.Bp, Ybar, np, v.sx, v.sx);
  add_out(p, v.gA, 1.0, 0.0, {});
  return G(v, one(p, (int)np));
}

// Ytot = Ybar2 Y^T + Y^T Ybar2 + Yd  (adjoint of Y2 = Y Y plus direct terms)
sincosm_status square_adjoint(Rev& v, const void* Ybar2, const void* YB, const void* Yd, void* out) {
  const int64_t np = v.m->np;
  Problem p = make_problem((int)v.r->n);
  add_seg(p, Ybar2, YB, np);
  add_seg(p, YB, Ybar2, np);
  add_in(p, Yd, np);
  add_out(p, T(out, *v.m), 1.0, 0.0, {1.0});
  return G(v, one(p, (int)np));
}

sincosm_status rev3(Rev& v) {
  const Modes& m = *v.m;
  const int64_t np = m.np;
  const int nv = (int)v.r->n;
  void* const* W = v.W;  // W0 Y, W1 V
  // Vbar = sx B Sbar -> Ybar2 = Cbar/24 + Vbar/120, Yd = -Cbar/2 - Vbar/6
  Problem p = make_problem(nv);
  add_seg(p, v.Bp, v.Sbar, np, v.sx, 1.0);
  add_in(p, v.Cbar, np);
  add_out(p, T(v.R[0], m), 1.0 / 120.0, 0.0, {1.0 / 24.0});
  add_out(p, T(v.R[1], m), -1.0 / 6.0, 0.0, {-0.5});
  SC_TRY(G(v, one(p, (int)np)));
  SC_TRY(square_adjoint(v, v.R[0], W[0], v.R[1], v.R[2]));
  return final_abar(v, W[1], v.R[2]);
}

sincosm_status rev4(Rev& v) {
  const Modes& m = *v.m;
  const int64_t np = m.np;
  const int nv = (int)v.r->n;
  void* const* W = v.W;  // W0 Y, W1 Y2, W2 W, W3 Pc, W4 V
  // Vbar -> R0, Ybar4 = Cbar + Vbar/7 -> R1
  Problem p = make_problem(nv);
  add_seg(p, v.Bp, v.Sbar, np, v.sx, 1.0);
  add_in(p, v.Cbar, np);
  add_out(p, T(v.R[0], m), 1.0, 0.0, {0.0});
  add_out(p, T(v.R[1], m), 1.0 / 7.0, 0.0, {1.0});
  SC_TRY(G(v, one(p, (int)np)));
  // Wbar = Y2^T Ybar4 -> R2;  Yd = -Wbar/720 - Cbar/2 - Vbar/6 -> R3
  p = make_problem(nv);
  add_seg(p, W[1], v.R[1], np);
  add_in(p, v.Cbar, np);
  add_in(p, v.R[0], np);
  add_out(p, T(v.R[2], m), 1.0, 0.0, {0.0, 0.0});
  add_out(p, T(v.R[3], m), -1.0 / 720.0, 0.0, {-0.5, -1.0 / 6.0});
  SC_TRY(G(v, one(p, (int)np)));
  // Ybar2 = Ybar4 W^T + Wbar/8! + Cbar/24 + Vbar/120 -> R4
  p = make_problem(nv);
  add_seg(p, v.R[1], W[2], np);
  add_in(p, v.R[2], np);
  add_in(p, v.Cbar, np);
  add_in(p, v.R[0], np);
  add_out(p, T(v.R[4], m), 1.0, 0.0, {1.0 / 40320.0, 1.0 / 24.0, 1.0 / 120.0});
  SC_TRY(G(v, one(p, (int)np)));
  SC_TRY(square_adjoint(v, v.R[4], W[0], v.R[3], v.R[5]));
  return final_abar(v, W[4], v.R[5]);
}

sincosm_status rev6(Rev& v) {
  const Modes& m = *v.m;
  const int64_t np = m.np;
  const int nv = (int)v.r->n;
  const Coeffs& k = coeffs();
  const double* x = k.x;
  const double* z = k.z6;
  void* const* W = v.W;  // W0 Y, W1 Y2, W2 W, W3 Y4, W4 L, W5 R, W6 Pc, W7 Q', W8 V
  // Vbar -> R0
  Problem p = make_problem(nv);
  add_seg(p, v.Bp, v.Sbar, np, v.sx, 1.0);
  add_out(p, T(v.R[0], m), 1.0, 0.0, {});
  SC_TRY(G(v, one(p, (int)np)));
  // Q'bar = Vbar Y4^T -> R1, Tbar = Cbar + z8 Q'bar + z4 Vbar -> R2 ; Y4u = Q'^T Vbar -> R3
  Problem p0 = make_problem(nv);
  add_seg(p0, v.R[0], W[3], np);
  add_in(p0, v.Cbar, np);
  add_in(p0, v.R[0], np);
  add_out(p0, T(v.R[1], m), 1.0, 0.0, {0.0, 0.0});
  add_out(p0, T(v.R[2], m), z[8], 0.0, {1.0, z[4]});
  Problem p1 = make_problem(nv);
  add_seg(p1, W[7], v.R[0], np);
  add_out(p1, T(v.R[3], m), 1.0, 0.0, {});
  SC_TRY(G(v, two(p0, p1, (int)np)));
  // Lbar = Tbar R^T -> R4 ; Rbar = L^T Tbar -> R5
  p0 = make_problem(nv);
  add_seg(p0, v.R[2], W[5], np);
  add_out(p0, T(v.R[4], m), 1.0, 0.0, {});
  p1 = make_problem(nv);
  add_seg(p1, W[4], v.R[2], np);
  add_out(p1, T(v.R[5], m), 1.0, 0.0, {});
  SC_TRY(G(v, two(p0, p1, (int)np)));
  // linear combination only: inputs Y4u, Lbar, Rbar, Tbar, Q'bar, Vbar
  p = make_problem(nv);
  add_in(p, v.R[3], np);
  add_in(p, v.R[4], np);
  add_in(p, v.R[5], np);
  add_in(p, v.R[2], np);
  add_in(p, v.R[1], np);
  add_in(p, v.R[0], np);
  add_out(p, T(v.R[6], m), 0.0, 0.0, {1.0, 1.0, x[7], 0.0, z[7], z[3]});   // Ybar4 total
  add_out(p, T(v.R[7], m), 0.0, 0.0, {0.0, x[3], x[6], x[8], z[6], z[2]}); // Ybar2 direct
  add_out(p, T(v.R[8], m), 0.0, 0.0, {0.0, 0.0, x[5], -0.5, z[5], z[1]});  // Ybar direct
  SC_TRY(G(v, one(p, (int)np)));
  // Wbar = Y2^T Ybar4 -> R2 ; Yd2 = Yd + x1 Wbar -> R8
  p = make_problem(nv);
  add_seg(p, W[1], v.R[6], np);
  add_in(p, v.R[8], np);
  add_out(p, T(v.R[2], m), 1.0, 0.0, {0.0});
  add_out(p, T(v.R[8], m), x[1], 0.0, {1.0});
  SC_TRY(G(v, one(p, (int)np)));
  // Ybar2 total = Ybar4 W^T + Ybar2d + x2 Wbar -> R7
  p = make_problem(nv);
  add_seg(p, v.R[6], W[2], np);
  add_in(p, v.R[7], np);
  add_in(p, v.R[2], np);
  add_out(p, T(v.R[7], m), 1.0, 0.0, {1.0, x[2]});
  SC_TRY(G(v, one(p, (int)np)));
  SC_TRY(square_adjoint(v, v.R[7], W[0], v.R[8], v.R[0]));
  return final_abar(v, W[8], v.R[0]);
}

sincosm_status rev7(Rev& v) {
  const Modes& m = *v.m;
  const int64_t np = m.np;
  const int nv = (int)v.r->n;
  const Coeffs& k = coeffs();
  const double(*a)[5] = k.a;
  const double* z = k.z7;
  void* const* W = v.W;  // W0 Y, W1 Y2, W2 C1, W3 L, W4 Y6, W5 C4, W6 V, W7 Q', W8 C
  // Vbar -> R0
  Problem p = make_problem(nv);
  add_seg(p, v.Bp, v.Sbar, np, v.sx, 1.0);
  add_out(p, T(v.R[0], m), 1.0, 0.0, {});
  SC_TRY(G(v, one(p, (int)np)));
  // Q'bar = Vbar C^T -> R1
  p = make_problem(nv);
  add_seg(p, v.R[0], W[8], np);
  add_out(p, T(v.R[1], m), 1.0, 0.0, {});
  SC_TRY(G(v, one(p, (int)np)));
  // Tbar (= C1bar) = Q'^T Vbar + Cbar + z11 Q'bar + z5 Vbar -> R2
  p = make_problem(nv);
  add_seg(p, W[7], v.R[0], np);
  add_in(p, v.Cbar, np);
  add_in(p, v.R[1], np);
  add_in(p, v.R[0], np);
  add_out(p, T(v.R[2], m), 1.0, 0.0, {1.0, z[11], z[5]});
  SC_TRY(G(v, one(p, (int)np)));
  // Lbar (= C2bar) = Tbar Y6^T -> R3
  p = make_problem(nv);
  add_seg(p, v.R[2], W[4], np);
  add_out(p, T(v.R[3], m), 1.0, 0.0, {});
  SC_TRY(G(v, one(p, (int)np)));
  // Kbar (= C3bar) = L^T Tbar + z10 Q'bar + z4 Vbar + Lbar -> R4
  p = make_problem(nv);
  add_seg(p, W[3], v.R[2], np);
  add_in(p, v.R[1], np);
  add_in(p, v.R[0], np);
  add_in(p, v.R[3], np);
  add_out(p, T(v.R[4], m), 1.0, 0.0, {z[10], z[4], 1.0});
  SC_TRY(G(v, one(p, (int)np)));
  // C4bar = Kbar C4^T + C4^T Kbar; epilogue: Ybar3, Ybar2 direct, Ybar direct from
  // C1bar = Tbar, C2bar = Lbar, C3bar = Kbar, C4bar, Pbar = Vbar, Qbar = Q'bar
  p = make_problem(nv);
  add_seg(p, v.R[4], W[5], np);
  add_seg(p, W[5], v.R[4], np);
  add_in(p, v.R[2], np);
  add_in(p, v.R[3], np);
  add_in(p, v.R[4], np);
  add_in(p, v.R[0], np);
  add_in(p, v.R[1], np);
  add_out(p, T(v.R[5], m), a[3][4], 0.0, {a[3][1], a[3][2], a[3][3], z[3], z[9]});
  add_out(p, T(v.R[6], m), a[2][4], 0.0, {a[2][1], a[2][2], a[2][3], z[2], z[8]});
  add_out(p, T(v.R[7], m), a[1][4], 0.0, {a[1][1], a[1][2], a[1][3], z[1], z[7]});
  SC_TRY(G(v, one(p, (int)np)));
  // Y3 = Y2 Y:  Ybar2 = Ybar3 Y^T + Ybar2d -> R6 ;  Ybar' = Y2^T Ybar3 + Ybard -> R7
  Problem p0 = make_problem(nv);
  add_seg(p0, v.R[5], W[0], np);
  add_in(p0, v.R[6], np);
  add_out(p0, T(v.R[6], m), 1.0, 0.0, {1.0});
  Problem p1 = make_problem(nv);
  add_seg(p1, W[1], v.R[5], np);
  add_in(p1, v.R[7], np);
  add_out(p1, T(v.R[7], m), 1.0, 0.0, {1.0});
  SC_TRY(G(v, two(p0, p1, (int)np)));
  SC_TRY(square_adjoint(v, v.R[6], W[0], v.R[7], v.R[8]));
  return final_abar(v, W[6], v.R[8]);
}

// Adjoint of one double-angle step from (Cbar', Sbar') to (Cbar, Sbar), with
// (SB, CB) the step's inputs computed on B = A^T; tmp is scratch.
sincosm_status rev_double_angle(Run& r, const Modes& m, const void* SB, const void* CB, const void* Cbn,
                                const void* Sbn, void* Cb, void* Sb, void* tmp) {
  const int64_t np = m.np;
  Problem p0 = make_problem((int)r.n);
  add_seg(p0, Cbn, SB, np, -2.0, 1.0);
  add_seg(p0, SB, Cbn, np, -2.0, 1.0);
  add_out(p0, internal(Sb, m, true), 1.0, 0.0, {});
  Problem p1 = make_problem((int)r.n);
  add_seg(p1, SB, Sbn, np, 2.0, 1.0);
  add_out(p1, internal(Cb, m, true), 1.0, 0.0, {});
  Problem p2 = make_problem((int)r.n);
  add_seg(p2, Sbn, CB, np, 2.0, 1.0);
  add_out(p2, internal(tmp, m, true), 1.0, 0.0, {});
  SC_TRY(gemm(r, Arith::F64, three(p0, p1, p2, (int)np), SINCOSM_TIMING_BACKWARD));
  Problem sum = make_problem((int)r.n);   // Sbar += tmp, element by element
  add_in(sum, Sb, np);
  add_in(sum, tmp, np);
  add_out(sum, internal(Sb, m, true), 0.0, 0.0, {1.0, 1.0});
  return gemm(r, Arith::F64, one(sum, (int)np), SINCOSM_TIMING_BACKWARD);
}

}  // namespace
}  // namespace sc

using namespace sc;

extern "C" {

size_t sincosm_backward_workspace_size(int64_t n, int dtype, int acc, int32_t s) {
  (void)acc;
  if (n <= 0 || dtype != SINCOSM_F64 || s < 0) return 0;
  Modes m;
  if (!modes_for(n, SINCOSM_F64, SINCOSM_PROD_NATIVE, m)) return 0;
  return bwd_layout(m, s).total;
}

sincosm_status sincosm_backward(int64_t n, int dtype, const void* A, int64_t lda, const void* Gc, int64_t ldgc,
                                const void* Gs, int64_t ldgs, void* gA, int64_t ldga, int acc, void* ws,
                                size_t ws_bytes, sincosm_plan* plan_host, void* stream_) {
  if (n < 0 || n > (1 << 20)) return SINCOSM_E_ARG;
  if (acc != SINCOSM_ACC_DOUBLE && acc != SINCOSM_ACC_SINGLE) return SINCOSM_E_ARG;
  if (dtype == SINCOSM_F32) return SINCOSM_E_UNSUPPORTED;
  if (dtype != SINCOSM_F64) return SINCOSM_E_ARG;
  if (n == 0) return SINCOSM_OK;
  if (!A || !gA || lda < n || ldga < n) return SINCOSM_E_ARG;
  if ((Gc && ldgc < n) || (Gs && ldgs < n)) return SINCOSM_E_ARG;
  if (overlaps(A, lda, gA, ldga, n, 8) || (Gc && overlaps(Gc, ldgc, gA, ldga, n, 8)) ||
      (Gs && overlaps(Gs, ldgs, gA, ldga, n, 8)))
    return SINCOSM_E_ARG;
  Modes m;
  if (!modes_for(n, SINCOSM_F64, SINCOSM_PROD_NATIVE, m)) return SINCOSM_E_ARG;
  const BwdLayout L0 = bwd_layout(m, 0);
  if (!ws || ws_bytes < L0.total || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  hipStream_t stream = (hipStream_t)stream_;
  char* base = (char*)ws;

  // plan of A (not of A^T): 1-norm of A, no copy
  const NormScratch ns = norm_scratch(base + L0.norm_off, m.np);
  SC_TRY(launch_norm_copy_plan(n, m.np, A, lda, true, nullptr, true, acc, ns, stream));
  sincosm_plan plan;
  SC_TRY(read_plan(ns.plan, &plan, stream, 1, "sincosm_backward", n));
  if (plan_host) *plan_host = plan;
  if (plan.status != SINCOSM_OK) {
    SC_TRY(launch_fill_nan(n, gA, ldga, true, stream));
    return SINCOSM_E_NONFINITE;
  }
  const int s = plan.s;
  const BwdLayout L = bwd_layout(m, s);
  if (ws_bytes < L.total) return SINCOSM_E_WORKSPACE;

  void* Bp = base + L.bp_off;
  SC_TRY(launch_transpose_pad(n, m.np, A, lda, true, Bp, true, stream));

  Run r;
  r.m = &m;
  r.n = n;
  r.Ap = Bp;
  for (int i = 0; i < 9; ++i) r.W[i] = base + L.w_off[i];
  r.stream = stream;
  void* Rb[9];
  for (int i = 0; i < 9; ++i) Rb[i] = base + L.rev_off[i];
  void* cot[4];
  for (int i = 0; i < 4; ++i) cot[i] = base + L.cot_off[i];
  const size_t mat = align_up((size_t)m.np * m.np * 8, 256);
  auto chainS = [&](int i) -> void* { return base + L.chain_off + mat * (size_t)(2 * i); };
  auto chainC = [&](int i) -> void* { return base + L.chain_off + mat * (size_t)(2 * i + 1); };

  // forward on B, keeping the scheme intermediates (W) and the double-angle inputs
  if (s > 0) {
    r.Cout = internal(chainC(0), m, true);
    r.Sout = internal(chainS(0), m, true);
  } else {  // the scheme's outputs are not needed by the reverse pass
    r.Cout = internal(Rb[0], m, true);
    r.Sout = internal(Rb[1], m, true);
  }
  const double sx = ldexp(1.0, -s);
  SC_TRY(run_scheme(r, plan.level, sx));
  for (int i = 0; i + 1 < s; ++i)
    SC_TRY(double_angle(r, chainS(i), chainC(i), internal(chainC(i + 1), m, true),
                        internal(chainS(i + 1), m, true)));

  // adjoints of the outputs, zero padded
  if (Gc) SC_TRY(launch_convert_pad(n, m.np, Gc, ldgc, true, cot[0], true, stream));
  else SC_TRY(launch_fill_zero(m.np, cot[0], true, stream));
  if (Gs) SC_TRY(launch_convert_pad(n, m.np, Gs, ldgs, true, cot[1], true, stream));
  else SC_TRY(launch_fill_zero(m.np, cot[1], true, stream));
  int cur = 0;  // (Cbar, Sbar) live in cot[2 cur], cot[2 cur + 1]
  for (int i = s - 1; i >= 0; --i) {
    const int nxt = cur ^ 1;
    SC_TRY(rev_double_angle(r, m, chainS(i), chainC(i), cot[2 * cur], cot[2 * cur + 1], cot[2 * nxt],
                            cot[2 * nxt + 1], Rb[0]));   // the scheme adjoint's buffers are free here
    cur = nxt;
  }

  Rev v;
  v.r = &r;
  v.m = &m;
  v.Bp = Bp;
  v.W = r.W;
  for (int i = 0; i < 9; ++i) v.R[i] = Rb[i];
  v.Cbar = cot[2 * cur];
  v.Sbar = cot[2 * cur + 1];
  v.gA = Target{gA, ldga, (int)n, true};
  v.sx = sx;
  switch (plan.level) {
    case 3: return rev3(v);
    case 4: return rev4(v);
    case 6: return rev6(v);
    default: return rev7(v);
  }
}

sincosm_status sincosm_backward_async(int64_t n, int dtype, const void* A, int64_t lda, const void* Gc,
                                      int64_t ldgc, const void* Gs, int64_t ldgs, void* gA, int64_t ldga, int acc,
                                      int32_t s_max, void* ws, size_t ws_bytes, sincosm_plan* plan_dev,
                                      void* stream_) {
  if (n < 0 || n > (1 << 20) || s_max < 0 || s_max > 1100) return SINCOSM_E_ARG;
  if (acc != SINCOSM_ACC_DOUBLE && acc != SINCOSM_ACC_SINGLE) return SINCOSM_E_ARG;
  if (dtype == SINCOSM_F32) return SINCOSM_E_UNSUPPORTED;
  if (dtype != SINCOSM_F64) return SINCOSM_E_ARG;
  if (n == 0) return SINCOSM_OK;
  if (!A || !gA || lda < n || ldga < n) return SINCOSM_E_ARG;
  if ((Gc && ldgc < n) || (Gs && ldgs < n)) return SINCOSM_E_ARG;
  if (overlaps(A, lda, gA, ldga, n, 8) || (Gc && overlaps(Gc, ldgc, gA, ldga, n, 8)) ||
      (Gs && overlaps(Gs, ldgs, gA, ldga, n, 8)))
    return SINCOSM_E_ARG;
  Modes m;
  if (!modes_for(n, SINCOSM_F64, SINCOSM_PROD_NATIVE, m)) return SINCOSM_E_ARG;
  const BwdLayout L = bwd_layout(m, s_max);
  if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  hipStream_t stream = (hipStream_t)stream_;
  char* base = (char*)ws;

  // plan of A (not of A^T) on the device, capped at s_max
  const NormScratch ns = norm_scratch(base + L.norm_off, m.np);
  SC_TRY(launch_norm_copy_plan(n, m.np, A, lda, true, nullptr, true, acc, ns, stream, 0, 1.0, s_max, plan_dev));
  void* Bp = base + L.bp_off;
  SC_TRY(launch_transpose_pad(n, m.np, A, lda, true, Bp, true, stream));

  Run r;
  r.m = &m;
  r.n = n;
  r.Ap = Bp;
  for (int i = 0; i < 9; ++i) r.W[i] = base + L.w_off[i];
  r.stream = stream;
  r.cond.plan = ns.plan;
  r.cond.level = 0;
  r.cond.step = -1;
  r.cond.select = 0;
  void* Rb[9];
  for (int i = 0; i < 9; ++i) Rb[i] = base + L.rev_off[i];
  void* cot[4];
  for (int i = 0; i < 4; ++i) cot[i] = base + L.cot_off[i];
  const size_t mat = align_up((size_t)m.np * m.np * 8, 256);
  auto chainS = [&](int i) -> void* { return base + L.chain_off + mat * (size_t)(2 * i); };
  auto chainC = [&](int i) -> void* { return base + L.chain_off + mat * (size_t)(2 * i + 1); };

  // forward on B as in sincosm_backward, every launch decided on the device:
  // the scheme's (C, S) go to the first double-angle inputs (or to scratch when
  // no step can run), forward step i runs while i + 1 < s
  if (s_max > 0) {
    r.Cout = internal(chainC(0), m, true);
    r.Sout = internal(chainS(0), m, true);
  } else {
    r.Cout = internal(Rb[0], m, true);
    r.Sout = internal(Rb[1], m, true);
  }
  SC_TRY(first_product(r, SCALE_2_POW_MINUS_S));
  r.y_ready = true;
  SC_TRY(enqueue_schemes_by_slot(r, acc));
  for (int i = 0; i + 1 < s_max; ++i) {
    r.cond.step = i + 1;
    SC_TRY(double_angle(r, chainS(i), chainC(i), internal(chainC(i + 1), m, true),
                        internal(chainS(i + 1), m, true)));
  }

  // adjoints of the outputs, zero padded, in pair 0; for odd s they move to
  // pair 1, where reverse step s - 1 reads them: step i reads pair (i + 1) & 1
  // and writes pair i & 1, so the scheme's adjoints end in pair 0 for every s
  if (Gc) SC_TRY(launch_convert_pad(n, m.np, Gc, ldgc, true, cot[0], true, stream));
  else SC_TRY(launch_fill_zero(m.np, cot[0], true, stream));
  if (Gs) SC_TRY(launch_convert_pad(n, m.np, Gs, ldgs, true, cot[1], true, stream));
  else SC_TRY(launch_fill_zero(m.np, cot[1], true, stream));
  SC_TRY(launch_copy_pair_if_odd(ns.plan, m.np, cot[0], cot[1], cot[2], cot[3], stream));
  for (int i = s_max - 1; i >= 0; --i) {
    r.cond.step = i;
    const int rd = (i + 1) & 1, wr = i & 1;
    SC_TRY(rev_double_angle(r, m, chainS(i), chainC(i), cot[2 * rd], cot[2 * rd + 1], cot[2 * wr],
                            cot[2 * wr + 1], Rb[0]));
  }
  r.cond.step = -1;

  // the reverse of each level's scheme, run only for the plan's level
  Rev v;
  v.r = &r;
  v.m = &m;
  v.Bp = Bp;
  v.W = r.W;
  for (int i = 0; i < 9; ++i) v.R[i] = Rb[i];
  v.Cbar = cot[0];
  v.Sbar = cot[1];
  v.gA = Target{gA, ldga, (int)n, true};
  v.sx = SCALE_2_POW_MINUS_S;
  r.cond.level = 3;
  SC_TRY(rev3(v));
  r.cond.level = 4;
  SC_TRY(rev4(v));
  r.cond.level = 6;
  SC_TRY(rev6(v));
  r.cond.level = 7;
  SC_TRY(rev7(v));
  return launch_fill_nan_if(ns.plan, n, gA, ldga, true, stream);
}

}  // extern "C"
