// Enqueue-only building blocks of the CG solver, shared by the synchronous
// cg_solve_normal and the request server (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "blas.h"
#include "wd_internal.h"

namespace wd {

// Offsets (bytes) of a CG workspace for `slots` right-hand sides. Where the
// iteration's vector work is fused into its applications of Q (nslices > 0),
// paps and rr hold the |Q p|^2 and <r,r> partial sums of the tile slices, and
// (FP32 arithmetic, where the update is fused too) A p is never stored, and p
// and p2 hold the search directions of two consecutive iterations (the x
// update of one iteration waits for the next, see CgEngine::chunk).
// With eo (an even-odd gauge field) the vectors are odd half fields of V/2
// sites, A = (gamma5 S)^2 with the odd-site Schur complement S, and e_lo /
// e_hi are the even half fields each application of gamma5 S passes through.
struct CgLayout {
  size_t bytes = 0;
  size_t r_hi = 0, t_hi = 0, x_lo = 0, r = 0, p = 0, p2 = 0, t = 0, ap = 0, partials = 0, pap = 0,
         scal = 0, rr = 0, paps = 0, e_lo = 0, e_hi = 0;
  int nslices = 0;
};
CgLayout cg_layout(const int32_t dims[4], int slots, int inner, bool eo = false);

size_t align256(size_t b);

// What the host does with a right-hand side after reading its scalars.
enum CgAction { kCgContinue, kCgRefresh, kCgNumeric };
// ... and after its true residual was recomputed.
enum CgOutcome { kCgKeepGoing, kCgConverged, kCgNotConverged, kCgFailed };

// sc: the kScalars doubles of one right-hand side.
CgAction cg_check(const double* sc, double tol, bool mixed, double delta, bool at_max);
CgOutcome cg_after_refresh(const double* sc, double tol, bool at_max);

// CG on D^dag D (or, with an even-odd gauge field, on S^dag S for the
// odd-site Schur complement S) for up to kMaxRhs slots that share one lattice
// and gauge field. Slot k's vectors are field k of each buffer: b and x (FP64 packed,
// caller- or server-owned) and the workspace. Every method only enqueues
// work on the stream and returns a wd_status.
class CgEngine {
 public:
  CgEngine(const wd_gauge* ghi, const wd_gauge* glo, int inner, int slots, const void* b, void* x,
           void* ws, hipStream_t st);

  void set_mass(int slot, double m) { masses_[slot] = m; }
  int inner() const { return inner_; }

  // scalars of the slots zeroed, <b,b>, x = 0 and r = b (or r = b - A x
  // when x0_given), inner residual and p = r.
  int start(const RhsSet& set, bool x0_given);
  // n CG iterations on the slots of set. Where the inner vector updates are
  // fused (FP32 arithmetic), the x update of an even-numbered iteration of
  // the chunk (0, 2, ...) that is not the last is left for the next one,
  // which applies both in turn (the same operations in the same order), with
  // that iteration's p kept in p2 meanwhile; a chunk ends with x and p
  // complete and p in its own buffer.
  int chunk(const RhsSet& set, int n);
  // (mixed precision: x += x_lo, x_lo = 0) FP64 true residual r = b - A x;
  // inner residual restarted from it
  int refresh(const RhsSet& set);
  // copies the scalars of every slot to host memory (async; pinned memory
  // for a true overlap)
  int fetch_scalars(double* host) const;

 private:
  // iteration j of a chunk of n
  int iterate(const RhsSet& set, int j, int n);
  // out = Q in (Q = gamma5 D, or gamma5 S through the even fields tmp)
  int apply_q(const wd_gauge* g, const double* m, const RhsSet& set, const void* in, void* tmp, void* out,
              const char* what) const;
  bool eo_ = false;
  const wd_gauge* ghi_;
  const wd_gauge* glo_;
  int inner_;
  int slots_;
  const void* b_;
  void* x_;
  void* ws_;
  hipStream_t st_;
  long V_ = 0, nhi_ = 0, nlo_ = 0, n32_ = 0;
  CgLayout lay_;
  double* partials_ = nullptr;
  double* rr_ = nullptr;
  double* paps_ = nullptr;
  double* pap_ = nullptr;
  double* scal_ = nullptr;
  double masses_[kMaxRhs] = {};
};

// The synchronous solver behind cg_solve_normal: all right-hand sides start
// together, the host checks the scalars every check_every iterations (into
// `host`, kMaxRhs * kScalars doubles, or a page-locked buffer of a pool when
// null) and recomputes true residuals as the engine asks. Arguments are
// checked by the caller.
int solve_sync(const wd_gauge* ghi, const wd_gauge* glo, const double* masses, int nrhs, const void* b,
               void* x, const wd_cg_params& prm, wd_cg_stats* stats, void* ws, hipStream_t caller,
               double* host);

}  // namespace wd
