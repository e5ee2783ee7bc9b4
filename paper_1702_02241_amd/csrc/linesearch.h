// Strong-Wolfe line search as a device-side state machine (one thread runs one
// step after every trial evaluation).  Included by the objective translation unit.
#pragma once

#include "rpca_internal.h"

namespace rpca_ls {

// Strong-Wolfe line search, one step of the state machine (Nocedal & Wright
// Alg. 3.5 bracketing + Alg. 3.6 zoom, cubic interpolation), run by one thread
// after each trial evaluation.

__device__ inline bool cubic_min(double a0, double f0, double d0, double a1, double f1, double d1,
                          double* out) {
  if (a0 == a1) return false;
  const double e1 = d0 + d1 - 3.0 * (f0 - f1) / (a0 - a1);
  const double disc = e1 * e1 - d0 * d1;
  if (!(disc >= 0.0) || !isfinite(disc)) return false;
  const double e2 = copysign(sqrt(disc), a1 - a0);
  const double den = d1 - d0 + 2.0 * e2;
  if (den == 0.0 || !isfinite(den)) return false;
  *out = a1 - (a1 - a0) * (d1 + e2 - e1) / den;
  return isfinite(*out);
}

__device__ inline void zoom_next(SolverState* st) {
  const double lo = st->a_lo, hi = st->a_hi;
  const double left = fmin(lo, hi), right = fmax(lo, hi), w = right - left;
  double a;
  if (!cubic_min(lo, st->f_lo, st->d_lo, hi, st->f_hi, st->d_hi, &a) || a < left + 0.01 * w ||
      a > right - 0.01 * w)
    a = 0.5 * (lo + hi);
  st->alpha = a;
}

__device__ inline void search_failed(SolverState* st) {
  if (st->count > 0 && !st->restarted) {
    // drop the memory once and retry along steepest descent
    st->count = 0;
    st->spare = 0;
    st->newest = -1;
    st->restarted = 1;
    st->phase = PH_DIRECTION;
  } else {
    st->stop = STOP_LINESEARCH;
    st->phase = PH_DONE;
  }
}

// Set up the line search along the direction d = -H g whose slope g^T d = gd is
// known (from the update's inner products, or from the direction pass).  g1 =
// ||g||_1 scales the very first step of a solve.  A non-descent direction drops
// the memory (steepest descent next) or, without memory, ends the solve.
// dir_pending: d still has to be formed by the direction pass of the next slot.
__device__ inline void setup_trial(SolverState* st, double gd, double g1, int dir_pending) {
  if (!(gd < 0.0) || !isfinite(gd)) {
    if (st->count > 0) {
      st->count = 0;
      st->spare = 0;
      st->newest = -1;
      st->phase = PH_DIRECTION;
    } else {
      st->stop = isfinite(gd) ? STOP_GTOL : STOP_NONFINITE;
      st->phase = PH_DONE;
    }
    st->dir_pending = 0;
    return;
  }
  st->dphi0 = gd;
  st->alpha = st->first_iter ? fmin(1.0, 1.0 / g1) : 1.0;
  st->first_iter = 0;
  st->ls_stage = 0;
  st->ls_trials = 0;
  st->a_prev = 0.0;
  st->f_prev = st->f;
  st->d_prev = gd;
  st->dir_pending = dir_pending;
  st->phase = PH_TRIAL;
}

__device__ inline void accept_trial(SolverState* st, double ft) {
  st->cur = 1 - st->cur;
  st->f = ft;
  st->restarted = 0;
  st->phase = PH_UPDATE;
}

__device__ inline void line_search_step(SolverState* st, double ft, double dt) {
  st->evals += 1;
  st->ls_trials += 1;
  st->f_t = ft;
  st->dphi_t = dt;
  const double a = st->alpha, f0 = st->f, d0 = st->dphi0, c1 = st->c1, c2 = st->c2;
  const bool finite = isfinite(ft) && isfinite(dt);
  // Approximate Wolfe (Hager & Zhang): once f-differences reach the rounding level of
  // the evaluation, accept a step whose slope satisfies
  // -c2|d0| <= dphi <= (1 - 2 c1)|d0| and whose value is within eps_f |f0| of f0.
  if (finite && ft <= f0 + st->eps_f * fabs(f0) && dt >= c2 * d0 && dt <= (2.0 * c1 - 1.0) * d0 &&
      ft > f0 + c1 * a * d0) {
    accept_trial(st, ft);
    return;
  }
  const bool armijo_fail = !finite || ft > f0 + c1 * a * d0;
  if (st->ls_stage == 0) {
    if (armijo_fail || (st->ls_trials > 1 && ft >= st->f_prev)) {
      st->a_lo = st->a_prev; st->f_lo = st->f_prev; st->d_lo = st->d_prev;
      st->a_hi = a; st->f_hi = finite ? ft : INFINITY; st->d_hi = finite ? dt : 0.0;
      st->ls_stage = 1;
      zoom_next(st);
    } else if (fabs(dt) <= -c2 * d0) {
      accept_trial(st, ft);
      return;
    } else if (dt >= 0.0) {
      st->a_lo = a; st->f_lo = ft; st->d_lo = dt;
      st->a_hi = st->a_prev; st->f_hi = st->f_prev; st->d_hi = st->d_prev;
      st->ls_stage = 1;
      zoom_next(st);
    } else {
      double an;
      const double lo_b = a + 0.01 * (a - st->a_prev), hi_b = 10.0 * a;
      if (!cubic_min(st->a_prev, st->f_prev, st->d_prev, a, ft, dt, &an) || an < lo_b || an > hi_b)
        an = fmin(fmax(2.0 * a, lo_b), hi_b);
      st->a_prev = a; st->f_prev = ft; st->d_prev = dt;
      st->alpha = an;
    }
  } else {
    if (armijo_fail || ft >= st->f_lo) {
      st->a_hi = a; st->f_hi = finite ? ft : INFINITY; st->d_hi = finite ? dt : 0.0;
    } else {
      if (fabs(dt) <= -c2 * d0) {
        accept_trial(st, ft);
        return;
      }
      if (dt * (st->a_hi - st->a_lo) >= 0.0) {
        st->a_hi = st->a_lo; st->f_hi = st->f_lo; st->d_hi = st->d_lo;
      }
      st->a_lo = a; st->f_lo = ft; st->d_lo = dt;
    }
    if (fabs(st->a_hi - st->a_lo) <= 1e-12 * fmax(1.0, fabs(st->a_hi))) {
      search_failed(st);
      return;
    }
    zoom_next(st);
  }
  if (st->ls_trials >= 30 || !(st->alpha > 0.0)) search_failed(st);
}


}  // namespace rpca_ls
