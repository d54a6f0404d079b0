#include "orth_estimate.h"

#include <algorithm>
#include <cmath>

namespace svt {

void OrthEstimate::reset(double unit, double root) {
  unit_ = unit;
  root_ = root;
  anorm_ = 0.0;
  alpha_.clear();
  beta_.assign(1, 0.0);
  mu_.clear();
  nu_.clear();
}

// A coefficient that is not positive and finite (a breakdown of the
// recurrence) leaves nothing to divide by: the new vector is taken as having
// lost its orthogonality entirely (level 1), never as NaN.
static bool usable(double c) { return c > 0.0 && std::isfinite(c); }

double OrthEstimate::push_u(double a, bool reorth) {
  const int j = (int)alpha_.size() + 1;  // u_j
  if (usable(a)) anorm_ = std::max(anorm_, a + beta_[(size_t)j - 1]);
  const double noise = usable(a) ? unit_ * root_ * anorm_ / a : 0.0;
  row_.assign((size_t)j - 1, usable(a) ? 0.0 : 1.0);
  double top = (usable(a) || j == 1) ? 0.0 : 1.0;
  for (int i = 1; i < j && usable(a); ++i) {
    // nu_ holds nu_{j,1..j-1}; mu_ holds mu_{j-1,1..j-2}
    const double nu_next = (i + 1 == j) ? 1.0 : nu_[(size_t)i];
    double t = beta_[(size_t)i] * nu_next + alpha_[(size_t)i - 1] * nu_[(size_t)i - 1];
    const double mu_old = (i == j - 1) ? 1.0 : mu_[(size_t)i - 1];
    t = (t - beta_[(size_t)j - 1] * mu_old) / a;
    t += std::copysign(noise, t);
    row_[(size_t)i - 1] = t;
    top = std::max(top, std::fabs(t));
  }
  alpha_.push_back(usable(a) ? a : 0.0);
  if (reorth) std::fill(row_.begin(), row_.end(), unit_);
  mu_.swap(row_);
  return top;
}

double OrthEstimate::push_v(double b, bool reorth) {
  const int j = (int)alpha_.size();  // v_{j+1}
  if (usable(b)) anorm_ = std::max(anorm_, alpha_[(size_t)j - 1] + b);
  const double noise = usable(b) ? unit_ * root_ * anorm_ / b : 0.0;
  row_.assign((size_t)j, usable(b) ? 0.0 : 1.0);
  double top = usable(b) ? 0.0 : 1.0;
  for (int i = 1; i <= j && usable(b); ++i) {
    // mu_ holds mu_{j,1..j-1}; nu_ holds nu_{j,1..j-1}
    double t = alpha_[(size_t)i - 1] * ((i == j) ? 1.0 : mu_[(size_t)i - 1]);
    if (i >= 2) t += beta_[(size_t)i - 1] * mu_[(size_t)i - 2];
    t -= alpha_[(size_t)j - 1] * ((i == j) ? 1.0 : nu_[(size_t)i - 1]);
    t /= b;
    t += std::copysign(noise, t);
    row_[(size_t)i - 1] = t;
    top = std::max(top, std::fabs(t));
  }
  beta_.push_back(usable(b) ? b : 0.0);
  if (reorth) std::fill(row_.begin(), row_.end(), unit_);
  nu_.swap(row_);
  return top;
}

void OrthEstimate::mark_u() { std::fill(mu_.begin(), mu_.end(), unit_); }
void OrthEstimate::mark_v() { std::fill(nu_.begin(), nu_.end(), unit_); }

void ReorthSchedule::start(double eta, double unit, double root, double growth_prior, int hold,
                           const std::vector<uint8_t> *replay, double replay_eta) {
  eta_ = eta;
  hold_ = hold;
  replay_eta_ = replay_eta;
  replay_.clear();
  if (replay != nullptr && replay->size() > (size_t)kReplayLead) {
    replay_.assign(replay->size() - (size_t)kReplayLead, 0);
    for (size_t h = 1; h < replay_.size(); ++h) replay_[h] = (*replay)[h + (size_t)kReplayLead];
  }
  unit_ = unit;
  verify_ = std::sqrt(unit);
  prior_ = std::max(growth_prior, kGrowthFloor);
  seen_ = 0.0;
  growth_ = prior_;
  // the rounding term alone, with |Y|_est / divisor taken as 2
  reset_level_ = unit * root * 2.0;
  est_.reset(unit, root);
  logs_.assign(kWindow, 0.0);
  nlogs_ = 0;
  sched_.clear();
  trig_.clear();
  level_.clear();
}

bool ReorthSchedule::decide(int h) {
  // vectors are decided in order, each once (a call out of order, which the
  // solver never makes, orthogonalises)
  if (h != (int)sched_.size()) return true;
  bool r = false, trig = false;
  double lev = reset_level_;
  if (h >= 1) {  // u_1 has no basis to be orthogonalised against
    const double pred = level_[(size_t)h - 1] * growth_;
    const bool replayed = h < (int)replay_.size();
    trig = pred > (replayed ? replay_eta_ : eta_) && h >= hold_;
    r = trig || trig_[(size_t)h - 1] || (replayed && replay_[(size_t)h]);
    lev = r ? reset_level_ : pred;
  }
  sched_.push_back(r ? 1 : 0);
  trig_.push_back(trig ? 1 : 0);
  level_.push_back(lev);
  return r;
}

void ReorthSchedule::repredict(int from) {
  for (int h = std::max(from, 2); h < (int)level_.size(); ++h)
    level_[(size_t)h] = sched_[(size_t)h] ? reset_level_ : level_[(size_t)h - 1] * growth_;
}

bool ReorthSchedule::advance(const double *alpha, const double *beta, int k) {
  bool ok = true;
  // only vectors already decided can be checked
  k = std::min(k, (int)sched_.size() / 2);
  while (est_.steps() < k) {
    const int j = est_.steps() + 1;
    for (int side = 0; side < 2; ++side) {
      const int h = 2 * (j - 1) + side;
      const bool r = sched_[(size_t)h] != 0;
      const double e = side == 0 ? est_.push_u(alpha[j - 1], r) : est_.push_v(beta[j], r);
      if (!r && e > verify_) ok = false;
      if (!r && h >= 2) {
        if (sched_[(size_t)h - 1]) {
          // the first vector after a reorthogonalised one: where levels restart
          reset_level_ = std::max(reset_level_, e / growth_);
        } else if (level_[(size_t)h - 1] > 0.0) {
          const double g = std::max(e, unit_) / level_[(size_t)h - 1];
          seen_ = std::max(seen_, g);
          logs_[(size_t)(nlogs_ % kWindow)] = std::log(std::max(g, 1.0));
          ++nlogs_;
        }
      }
      // an orthogonalised vector's row is u, but its successor starts from
      // the rounding term: predictions continue from the restart level
      level_[(size_t)h] = r ? reset_level_ : std::max(e, unit_);
    }
  }
  if (nlogs_ >= kWindow) {
    double mean = 0.0;
    for (int i = 0; i < kWindow; ++i) mean += logs_[(size_t)i];
    growth_ = std::max(kGrowthFloor, kSafety * std::exp(mean / kWindow));
  } else {
    growth_ = std::max(prior_, seen_);
  }
  repredict(2 * est_.steps());
  return ok;
}

int first_trigger(const double *alpha, const double *beta, int k, double eta, double unit, double root) {
  OrthEstimate est;
  est.reset(unit, root);
  for (int j = 1; j <= k; ++j) {
    if (est.push_u(alpha[j - 1], false) > eta) return 2 * (j - 1);
    if (est.push_v(beta[j], false) > eta) return 2 * j - 1;
  }
  return 2 * k;
}

std::vector<uint8_t> exact_pattern(const double *alpha, const double *beta, int k, double eta, double unit,
                                   double root) {
  std::vector<uint8_t> pat((size_t)(2 * std::max(k, 0)), 0);
  OrthEstimate est;
  est.reset(unit, root);
  bool force = false;
  for (int j = 1; j <= k; ++j) {
    // u_j (u_1 has no basis)
    double e = est.push_u(alpha[j - 1], false);
    bool d = j > 1 && (e > eta || force);
    force = false;
    if (d) {
      est.mark_u();
      pat[(size_t)(2 * (j - 1))] = 1;
      force = e > eta;
    }
    // v_{j+1}
    e = est.push_v(beta[j], false);
    d = e > eta || force;
    force = false;
    if (d) {
      est.mark_v();
      pat[(size_t)(2 * j - 1)] = 1;
      force = e > eta;
    }
  }
  return pat;
}

}  // namespace svt
