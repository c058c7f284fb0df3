// Device-resident scalars and the small-kernel launchers (internal).
#pragma once

#include "common.h"

namespace yand {

// Scalars of one solve, kept on the device and read back once per iteration.
struct DevScalars {
  double f;          // objective at the current point
  double gn;         // |projected gradient|
  double mux;        // mu^T x
  double mom[4];     // m1..m4
  double tr;         // trace of B
  double gamma;      // scale of the (I - P_S) block of M
  double tang_scale; // mean diagonal of the tangent Hessian
  double lambda;     // absolute regularisation
  double GE[9];      // E^T B E
  double mud;        // mu^T d
  double coef[5];    // A0..A4
  double amax;       // feasibility cap
  double alpha;      // chosen step
  double aux[4];     // PCG dots
  int status;        // quartic step status (0 or -6)
  int fail;          // Cholesky pivot failure
  int nonfinite;     // NaN/Inf seen
  int nhold;         // coordinates the face solver holds at the bound
  int done;          // |G| <= eps at this iteration: the rest is skipped
  int frozen;        // lane stopped by the host: every pass is skipped
  double kkt;        // projected-simplex KKT residual (simplex set)
  double nfree;      // free coordinates of the current face (simplex set)
  int projected;     // this iteration took the projected trial segment
  int release;       // drop the holds at the next face evaluation
  int ptbad;         // push-through trace not applicable (psi'' = 0, lambda 0)
  int cgdone;        // PCG: converged or broke down, later steps skipped
  int cgit;          // PCG: iterations taken
  int lsskip;        // skip the raw line search (done, or segment taken)
  int segskip;       // skip the projected-segment trial (no candidate)
  double mudseg;     // mu^T dbar of the projected segment
  int nhold0;        // holds after this iteration's face evaluation
  int sneg;          // push-through trace: bars with psi''(z_t) < 0
};

// Face masks: mask[j] = 1 for a free coordinate of the current face of
// Delta(tau), 0 for a bound one; nullptr means every coordinate is free
// (affine budget set).  With a mask the first frame column E[0] holds
// mask / sqrt(nfree), and the projector P_S = diag(mask) - sum_a e_a e_a^T.

// eps < 0: never mark done.  Also clears fail and status for the iteration.
hipError_t launch_grad_project(const double* g, double* E, int p0, int64_t n,
                               DevScalars* sc, hipStream_t st,
                               double eps = -1.0,
                               const double* mask = nullptr);
hipError_t launch_trace_scale(const double* B, int64_t ld, int64_t n,
                              const double* E, const double* W, int p,
                              double reg, DevScalars* sc, hipStream_t st,
                              const double* mask = nullptr);
hipError_t launch_project(const double* B, double* M, int64_t ld, int64_t n,
                          int64_t np, const double* E, const double* W, int p,
                          const DevScalars* sc, hipStream_t st,
                          const double* mask = nullptr);
hipError_t launch_trace_weight(const double* rn, int nt, int64_t Tp,
                               const double* AE, int p, const DevScalars* sc,
                               double* q, hipStream_t st);
// mp1 < 0: take m + 1 from the face (nfree - p + 2).
hipError_t launch_rhs(const double* Bnu, const double* t3, const double* E,
                      int p, int64_t n, double mp1, const DevScalars* sc,
                      double* r, hipStream_t st, const double* mask = nullptr);
hipError_t launch_direction(const double* y, const double* E, int p,
                            int64_t n, const double* x, const double* mu,
                            double tau, int simplex, double* d,
                            DevScalars* sc, hipStream_t st,
                            const double* mask = nullptr);
// Face of Delta(tau) at x: mask, E[0] = mask / sqrt(nfree), sc->nfree.
hipError_t launch_face(const double* x, const double* g, int64_t n, double tau,
                       double* E, double* mask, double* hold, DevScalars* sc,
                       hipStream_t st);
// hold[j] = 0 for every j, sc->nhold = sc->release = 0.
hipError_t launch_reset_hold(double* hold, int64_t n, DevScalars* sc,
                             hipStream_t st);
// sc->kkt = |x - Pi_Delta(tau)(x - g)|_2; done when kkt <= eps (eps >= 0).
// tmp: n doubles.
hipError_t launch_kkt(const double* x, const double* g, int64_t n, double tau,
                      double eps, double* tmp, DevScalars* sc, hipStream_t st);
// Boundary block, first part: sets sc->lsskip = done, sc->segskip = 1;
// when sc->amax < eta, forms the corrected segment dbar =
// Pi_{Delta(tau)}(x + eta d) - x in tmp; if it is a nonzero descent
// direction it becomes the candidate (segskip = 0, mudseg = mu^T dbar),
// otherwise the face solver takes over (launch_hold semantics).  tmp: n.
hipError_t launch_boundary(const double* x, const double* g, const double* mu,
                           int64_t n, double tau, double eta, double* d,
                           double* tmp, const double* mask, double* hold,
                           DevScalars* sc, hipStream_t st);
// Boundary block, second part (skipped while segskip): the segment's quartic
// from the line-pass sums and its step over [0, 1] with the chosen rule; a
// step of at least kSegmentUsable takes the segment (d = dbar, coefficients
// and step kept, lsskip = 1, projected set); otherwise the face solver holds
// the released bound coordinates that d drives down and the coordinates
// that stop the raw step at alpha_max (hold[j] = 1, nhold counts them).
hipError_t launch_segment_decide(const double* sums, double invT, Coef c,
                                 int select, const double* x, int64_t n,
                                 double tau, double* d, const double* tmp,
                                 const double* mask, double* hold,
                                 DevScalars* sc, hipStream_t st);
// out = Pi_{Delta(tau)}(y) (one workgroup).
hipError_t launch_project_simplex(const double* y, int64_t n, double tau,
                                  double* out, hipStream_t st);
// dst[i] = src[i] unless *skip; fill dst with v unless *skip.
hipError_t launch_copy(double* dst, const double* src, int64_t count,
                       hipStream_t st, const int* skip = nullptr);
hipError_t launch_fill(double* dst, int64_t count, double v, hipStream_t st,
                       const int* skip = nullptr);
hipError_t launch_coef_step(const double* sums, double invT, Coef c,
                            int select, DevScalars* sc, hipStream_t st,
                            const int* skip = nullptr);
hipError_t launch_select_step(DevScalars* sc, hipStream_t st);
hipError_t launch_objective(const double* sums, double invT, Coef c,
                            DevScalars* sc, hipStream_t st);
hipError_t launch_dot(const double* u, const double* v, int64_t n, double* out,
                      hipStream_t st);
hipError_t launch_axpy(double* x, const double* d, int64_t n,
                       const DevScalars* sc, hipStream_t st);

}  // namespace yand
