// Partial reorthogonalisation of the bidiagonalisation (Section 5.1.1: the
// partial SVD of each iterate by Lanczos bidiagonalisation with partial
// reorthogonalisation).  Host code only.
//
// The bidiagonalisation alpha_j u_j = Y v_j - beta_j u_{j-1}, beta_{j+1}
// v_{j+1} = Y^T u_j - alpha_j v_j loses orthogonality in floating point as
// Ritz values converge.  Taking the inner products of the two relations with
// u_i and v_i and using the relations of step i gives, for the levels mu_{j,i}
// = u_j^T u_i and nu_{j,i} = v_j^T v_i (i < j; 1 on the diagonal),
//
//   alpha_j mu_{j,i}      = beta_{i+1} nu_{j,i+1} + alpha_i nu_{j,i} - beta_j mu_{j-1,i}
//   beta_{j+1} nu_{j+1,i} = alpha_i mu_{j,i} + beta_i mu_{j,i-1} - alpha_j nu_{j,i}
//
// up to the rounding of step j.  OrthEstimate runs these on the coefficients
// alone (the recurrences of Simon for symmetric Lanczos and of Larsen for
// bidiagonalisation), adding the rounding as u c |Y|_est / divisor with the
// sign of the value (u: the unit roundoff of the stored vectors; |Y|_est: the
// largest alpha_i + beta_i so far; c: sqrt(m + n) for FP64 vectors, 1 for
// FP32 vectors, whose rounding is dominated by that of their storage, which
// has no systematic direction).  A vector orthogonalised against its whole
// basis has its row set to u.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace svt {

class OrthEstimate {
 public:
  void reset(double unit, double root);
  // u_j (j = steps() + 1) with coefficient alpha_j: returns the largest
  // |mu_{j,i}|, i < j, as the recurrence gives it; reorth: u_j was then
  // orthogonalised against u_1 .. u_{j-1} (its row becomes u).
  double push_u(double alpha_j, bool reorth);
  // v_{j+1} (j = steps()) with coefficient beta_{j+1}: the largest
  // |nu_{j+1,i}|, i <= j; reorth as for push_u.
  double push_v(double beta_next, bool reorth);
  // the latest u (v) taken as orthogonalised after all: its row becomes u
  void mark_u();
  void mark_v();
  int steps() const { return (int)alpha_.size(); }
  double unit() const { return unit_; }

 private:
  double unit_ = 0.0, root_ = 0.0, anorm_ = 0.0;
  std::vector<double> alpha_;   // alpha_[j - 1] = alpha_j
  std::vector<double> beta_;    // beta_[j - 1] = beta_j; beta_1 multiplies u_0 = 0
  std::vector<double> mu_, nu_; // the rows of the latest u and v
  std::vector<double> row_;
};

// The schedule of partial reorthogonalisation for one bidiagonalisation run
// whose coefficients reach the host only some steps after the device has
// taken them.  Vector h is the one made by half-step h (h = 2(j - 1): u_j; h
// = 2j - 1: v_{j+1}).  Before a half-step is launched, decide(h) predicts the
// level of its vector as the previous vector's level times a growth factor
// per half-step and orthogonalises it when the prediction passes eta, and
// then also the next vector (of the other side).  An orthogonalised vector's
// successor restarts from the rounding term, not from u: its predicted level
// is a restart level times the growth.  When coefficients arrive, advance()
// runs OrthEstimate on them with the schedule that was applied: levels up to
// there become exact, the growth factor becomes 1.25 times the geometric mean
// of the last 8 ratios between consecutive levels of vectors left alone
// (before 8 are seen, the largest ratio seen, and at least the value carried
// from the previous run), the restart level the largest seen (divided by the
// growth), and a vector left alone whose level
// passed `verify` (semi-orthogonality, sqrt(u)) is reported so the caller
// can start again with full reorthogonalisation.
class ReorthSchedule {
 public:
  // hold: no vector before this half-step is orthogonalised on a prediction
  // (the replayed first trigger of the previous bidiagonalisation, less a
  // margin; 0: none).  replay (may be null): the vectors the exact policy
  // orthogonalised in the previous bidiagonalisation (exact_pattern); each
  // is orthogonalised here kReplayLead half-steps earlier, and over the
  // pattern's length a prediction must pass replay_eta (not eta) to add one.
  void start(double eta, double unit, double root, double growth_prior, int hold = 0,
             const std::vector<uint8_t> *replay = nullptr, double replay_eta = 0.0);
  bool decide(int h);
  // alpha_1..alpha_k and beta_1..beta_{k+1} (beta[0] = beta_1, unused):
  // returns false if an unreorthogonalised vector passed `verify`.
  bool advance(const double *alpha, const double *beta, int k);
  bool reorthogonalised(int h) const { return h < (int)sched_.size() && sched_[(std::size_t)h]; }
  double growth() const { return growth_; }
  double growth_seen() const { return seen_; }
  double verify() const { return verify_; }
  int exact_vectors() const { return 2 * est_.steps(); }

  static constexpr double kGrowthFloor = 1.5;
  static constexpr int kWindow = 8;         // ratios in the sustained growth
  static constexpr double kSafety = 1.25;   // on the sustained growth
  static constexpr int kReplayLead = 2;     // half-steps ahead of the replayed pattern

 private:
  void repredict(int from);
  OrthEstimate est_;
  double eta_ = 0.0, verify_ = 0.0, unit_ = 0.0, replay_eta_ = 0.0;
  int hold_ = 0;
  std::vector<uint8_t> replay_; // vector h orthogonalised as the replayed pattern says
  double growth_ = kGrowthFloor, seen_ = 0.0, prior_ = 0.0;
  double reset_level_ = 0.0;    // predicted level of a vector just orthogonalised
  std::vector<double> logs_;    // logs of the last kWindow ratios
  int nlogs_ = 0;
  std::vector<uint8_t> sched_;  // vector h orthogonalised against its basis
  std::vector<uint8_t> trig_;   // ... because its own prediction passed eta
  std::vector<double> level_;   // level after vector h (exact below exact_vectors())
};

// The exact policy replayed on the coefficients of a finished
// bidiagonalisation (alpha_1..alpha_k, beta[j] = beta_{j+1}): the first
// half-step at which the estimate of a vector, with nothing orthogonalised
// before it, passes eta; 2k if none does.  Consecutive SVT iterates put it
// within a few half-steps of each other.
int first_trigger(const double *alpha, const double *beta, int k, double eta, double unit, double root);

// The whole exact policy replayed the same way: pattern[h] = 1 for each
// vector h (of 2k) it orthogonalises, a vector whose estimate passes eta and
// the next vector after it.
std::vector<uint8_t> exact_pattern(const double *alpha, const double *beta, int k, double eta, double unit,
                                   double root);

}  // namespace svt
