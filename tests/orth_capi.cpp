// A C interface to the library's partial-reorthogonalisation estimate and
// schedule (orth_estimate.cpp), for CPU tests through ctypes.
#include <cstdint>
#include <vector>

#include "orth_estimate.h"

extern "C" {

void *est_new(double unit, double root) {
  auto *e = new svt::OrthEstimate();
  e->reset(unit, root);
  return e;
}
double est_push_u(void *e, double a, int reorth) { return static_cast<svt::OrthEstimate *>(e)->push_u(a, reorth != 0); }
double est_push_v(void *e, double b, int reorth) { return static_cast<svt::OrthEstimate *>(e)->push_v(b, reorth != 0); }
void est_free(void *e) { delete static_cast<svt::OrthEstimate *>(e); }

void *sched_new(double eta, double unit, double root, double prior, int hold) {
  auto *s = new svt::ReorthSchedule();
  s->start(eta, unit, root, prior, hold);
  return s;
}
void *sched_new_replay(double eta, double unit, double root, double prior, int hold, const uint8_t *pattern,
                       int npattern, double replay_eta) {
  auto *s = new svt::ReorthSchedule();
  std::vector<uint8_t> pat(pattern, pattern + npattern);
  s->start(eta, unit, root, prior, hold, &pat, replay_eta);
  return s;
}
int exact_pattern(const double *alpha, const double *beta, int k, double eta, double unit, double root,
                  uint8_t *out) {
  const std::vector<uint8_t> p = svt::exact_pattern(alpha, beta, k, eta, unit, root);
  for (size_t h = 0; h < p.size(); ++h) out[h] = p[h];
  return (int)p.size();
}
int first_trigger(const double *alpha, const double *beta, int k, double eta, double unit, double root) {
  return svt::first_trigger(alpha, beta, k, eta, unit, root);
}
int sched_decide(void *s, int h) { return static_cast<svt::ReorthSchedule *>(s)->decide(h) ? 1 : 0; }
int sched_advance(void *s, const double *alpha, const double *beta, int k) {
  return static_cast<svt::ReorthSchedule *>(s)->advance(alpha, beta, k) ? 1 : 0;
}
double sched_growth(void *s) { return static_cast<svt::ReorthSchedule *>(s)->growth(); }
double sched_growth_seen(void *s) { return static_cast<svt::ReorthSchedule *>(s)->growth_seen(); }
void sched_free(void *s) { delete static_cast<svt::ReorthSchedule *>(s); }

}  // extern "C"
