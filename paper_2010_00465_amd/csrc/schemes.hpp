// Launch-sequence builders shared by the forward, batched and reverse passes.
#pragma once

#include <initializer_list>

#include "common.hpp"

namespace sc {

struct Target {
  void* p;
  int64_t ld;
  int lim;
  bool f64;
};

struct Modes {
  Arith poly, sq;
  bool poly_f64, sq_f64, user_f64;
  int tile;
  int64_t np;
};

struct Layout {
  size_t norm_off, ap_off, w_off[9], q_off[4], i8_off, total;   // i8_off: operand slices (I8X5 only)
};

struct Recorder;   // captures launches instead of enqueuing them (batched templates)

struct Run {
  const Modes* m;
  int64_t n;
  const void* Ap;
  void* W[9];
  Target Cout, Sout;   // where the scheme's C and S go (squaring input or user buffers)
  hipStream_t stream;
  Recorder* rec = nullptr;
  bool y_ready = false;   // W0 already holds Y = (2^-s A)^2: the schemes skip their first product
  bool timed = true;      // launch timing may record events (off where nothing may be allocated)
  DevCond cond{};         // copied into every launch (plan == nullptr: launches always run)
  void* i8ws = nullptr;   // operand-slice scratch of I8X5 products
};

// Launch capture used to build the batched path's stage templates from the
// same scheme builders: buffers are symbolic ids encoded as small pointers.
struct Recorder {
  GemmLaunch launches[8];
  int count = 0;
};

Problem make_problem(int nvalid);
void add_seg(Problem& p, const void* L, const void* R, int64_t ld, double lsc = 1.0, double rsc = 1.0);
void add_in(Problem& p, const void* m, int64_t ld);
void add_out(Problem& p, const Target& t, double e, double d, std::initializer_list<double> c);
GemmLaunch one(const Problem& p, int np);
GemmLaunch two(const Problem& p0, const Problem& p1, int np);
GemmLaunch three(const Problem& p0, const Problem& p1, const Problem& p2, int np);
bool modes_for(int64_t n, int dtype, int prod, Modes& m);
Layout layout_for(const Modes& m);
// Copy `count` plan records from the device and wait for them; with SINCOSM_LOG
// set, the first is printed to stderr tagged with `who` and n.
sincosm_status read_plan(const sincosm_plan* dev, sincosm_plan* host, hipStream_t stream, int count = 1,
                         const char* who = nullptr, int64_t n = 0);
bool overlaps(const void* a, int64_t lda, const void* b, int64_t ldb, int64_t n, size_t es);
Target internal(void* p, const Modes& m, bool f64);
sincosm_status gemm(Run& r, Arith ar, const GemmLaunch& g, int kind = -1);
// G1 of every scheme: Y = (sx A)(sx A) into W0 (skipped when r.y_ready).
sincosm_status first_product(Run& r, double sx);
sincosm_status scheme3(Run& r, double sx);
sincosm_status scheme4(Run& r, double sx);
sincosm_status scheme5(Run& r, double sx);
sincosm_status scheme6(Run& r, double sx);
sincosm_status scheme7(Run& r, double sx);
sincosm_status run_scheme(Run& r, int level, double sx);
sincosm_status double_angle(Run& r, const void* Sc, const void* Cc, const Target& Cn, const Target& Sn);
// Device-planned calls: the launch sequences of several schemes (fn(r, level)
// for each of `levels`) packed into slot launches whose workgroups compute
// the problem of the plan's level (r.cond.plan set).
typedef sincosm_status (*SchemeFn)(Run& r, int level);
sincosm_status enqueue_by_slot(Run& r, const int* levels, int nlev, SchemeFn fn);
// The products of the cos/sin schemes after the shared first one (r.y_ready set).
sincosm_status enqueue_schemes_by_slot(Run& r, int acc);
// Shared by sincosm_eval_async and sincosm_expi_eval_async: the padded copy of
// pre * A with its device plan (s capped by s_max), the schemes and s_max
// guarded double-angle steps, leaving the pair in the ping-pong buffers
// (q1, q0) for even s and (q3, q2) for odd s. Returns the plan record.
sincosm_status enqueue_async_pair(Run& r, const Layout& L, char* base, const void* A, int64_t lda, int acc,
                                  double pre, int s_max, sincosm_plan* plan_dev, const sincosm_plan** plan_rec);
// Body of sincosm_eval_planned on a given workspace (timed = false: no launch
// timing events, so nothing is allocated).
sincosm_status eval_planned(int64_t n, int dtype, const void* A, int64_t lda, void* C, int64_t ldc, void* S,
                            int64_t lds, int acc, int prod, const sincosm_plan* plan_in, void* ws,
                            size_t ws_bytes, sincosm_plan* plan_dev, hipStream_t stream, bool timed);

}  // namespace sc
