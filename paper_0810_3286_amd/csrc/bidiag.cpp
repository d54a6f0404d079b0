// Host SVD of an upper-bidiagonal matrix by implicit-shift QR.
//
// Invariant kept throughout: B_input = P * B_current * Q^T.  A rotation G
// applied to rows (a, b) of B_current is undone by P <- P G^T; a rotation H
// applied to columns (a, b) is undone by Q <- Q H.  When B_current is
// diagonal, its (sign-corrected) diagonal holds the singular values.  Only
// the last row of P is accumulated (for the residual bounds) and the right
// rotations are logged; the vectors that are needed are formed afterwards
// (bidiag_vectors).
//
// The QR sweep is the Golub-Kahan step: a shift mu from the trailing 2 x 2 of
// B^T B (the eigenvalue nearer its last diagonal entry), a first right
// rotation chosen from (d0^2 - mu, d0 e0), and a bulge chased to the bottom by
// alternating left and right rotations.  A zero diagonal entry splits the
// problem after rotating its superdiagonal neighbour away.  On longer blocks
// two sweeps run at once, one with each eigenvalue of that 2 x 2 as its
// shift, the second bulge a few columns behind the first: a sweep is one
// long chain of dependent square roots and divisions, and two independent
// chains take about the time of one (about 15% more rotations in all, at
// half the time each).
//
// Both parts are host work that the device waits for, so each is compiled
// twice, for the baseline x86-64 target and with AVX2 and FMA, and the
// second is taken where the processor has them.  The QR sweep is a chain of
// dependent square roots and divisions (FMA shortens it); the vectors are
// independent of each other and are taken a block of columns at a time.
#include "bidiag.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

namespace svt {

namespace {

constexpr double kEps = 2.220446049250313e-16;
constexpr int kPairMin = 16;  // blocks of at least this many columns take paired sweeps
constexpr int kPairLag = 3;   // columns between the two bulges

struct Rot {
  double c, s, r;
};

// sqrt(a^2 + b^2): the plain formula where the squares can neither overflow
// nor underflow (it is within an ulp of the exact value), hypot elsewhere --
// hypot's scaling makes it several times slower, and the rotations of the
// implicit QR are most of the host work of a convergence check.
__attribute__((always_inline)) inline double norm2(double a, double b) {
  const double m = std::max(std::fabs(a), std::fabs(b));
  if (m > 1e-150 && m < 1e150) return std::sqrt(a * a + b * b);
  return std::hypot(a, b);
}

// c, s with -s*a + c*b = 0 and c*a + s*b = r >= 0 (r = sqrt(a^2 + b^2)).
__attribute__((always_inline)) inline Rot make_rot(double a, double b) {
  if (b == 0.0) return {a >= 0.0 ? 1.0 : -1.0, 0.0, std::fabs(a)};
  const double r = norm2(a, b);
  return {a / r, b / r, r};
}

struct Acc {
  std::vector<BidiagRot> *rots;  // right rotations, in order
  std::vector<double> *plast;    // last row of P

  // Only the last row of P is accumulated (the residual bounds need it); the
  // vectors are formed afterwards from the log of right rotations.
  // P <- P G^T for G acting on rows (a, b): new_a = c a + s b, new_b = -s a + c b.
  __attribute__((always_inline)) void left(int a, int b, double c, double s) {
    double &x = (*plast)[a], &y = (*plast)[b];
    const double xa = x, yb = y;
    x = c * xa + s * yb;
    y = -s * xa + c * yb;
  }
  // Q <- Q H for H acting on columns (a, b): new_a = c a + s b, new_b = -s a + c b.
  __attribute__((always_inline)) void right(int a, int b, double c, double s) { rots->push_back({a, b, c, s}); }
};

bool have_avx2_fma() {
  static const bool yes = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
  return yes;
}

__attribute__((always_inline)) inline bool svd_core(const std::vector<double> &d_in,
                                                    const std::vector<double> &e_in, BidiagSVD &out) {
  const int k = (int)d_in.size();
  out.sigma.assign(k, 0.0);
  out.p_last.assign(k, 0.0);
  out.P.clear();
  out.Q.clear();
  out.nvec = 0;
  out.rots.clear();
  out.src.assign(k, 0);
  out.sgn.assign(k, 1);
  if (k == 0) return true;
  std::vector<double> d(d_in), e(k > 1 ? k - 1 : 0, 0.0);
  for (int i = 0; i + 1 < k; ++i) e[i] = e_in[i];
  out.p_last[k - 1] = 1.0;
  Acc acc{&out.rots, &out.p_last};

  for (int i = 0; i < k; ++i)
    if (!std::isfinite(d[i])) return false;
  for (int i = 0; i + 1 < k; ++i)
    if (!std::isfinite(e[i])) return false;
  double bnorm = 0.0;
  for (int i = 0; i < k; ++i) bnorm = std::max(bnorm, std::fabs(d[i]));
  for (int i = 0; i + 1 < k; ++i) bnorm = std::max(bnorm, std::fabs(e[i]));
  const double abs_tol = kEps * bnorm;

  // implicit-shift QR needs about two sweeps per singular value
  const long max_sweeps = 30L * k + 1000;
  long sweeps = 0;
  int hi = k - 1;
  while (hi > 0) {
    // deflate negligible superdiagonals
    for (int i = 0; i < hi; ++i)
      if (std::fabs(e[i]) <= kEps * (std::fabs(d[i]) + std::fabs(d[i + 1])) || std::fabs(e[i]) <= abs_tol)
        e[i] = 0.0;
    while (hi > 0 && e[hi - 1] == 0.0) --hi;
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++sweeps > max_sweeps) return false;

    // a (numerically) zero diagonal entry in the block: rotate its
    // superdiagonal neighbour out and split
    int zero_at = -1;
    for (int i = lo; i <= hi; ++i)
      if (std::fabs(d[i]) <= abs_tol) { zero_at = i; break; }
    if (zero_at >= 0) {
      const int i = zero_at;
      d[i] = 0.0;
      if (i < hi) {
        // chase B[i][j] along row i with left rotations on rows (i, j)
        double f = e[i];
        e[i] = 0.0;
        for (int j = i + 1; j <= hi; ++j) {
          const Rot g = make_rot(d[j], f);  // new_j = c row_j + s row_i, new_i = c row_i - s row_j
          d[j] = g.r;
          // rows (j, i): new_j = c j + s i ; new_i = -s j + c i
          acc.left(j, i, g.c, g.s);
          if (j < hi) {
            f = -g.s * e[j];
            e[j] = g.c * e[j];
          }
        }
      } else {
        // last diagonal zero: chase B[j][hi] up column hi with right rotations
        double f = e[hi - 1];
        e[hi - 1] = 0.0;
        for (int j = hi - 1; j >= lo; --j) {
          const Rot g = make_rot(d[j], f);  // cols (j, hi): new_j = c j + s hi ; new_hi = -s j + c hi
          d[j] = g.r;
          acc.right(j, hi, g.c, g.s);
          if (j > lo) {
            f = -g.s * e[j - 1];
            e[j - 1] = g.c * e[j - 1];
          }
        }
      }
      continue;
    }

    // Golub-Kahan step on d[lo..hi], e[lo..hi-1]
    const double dm = d[hi - 1], dn = d[hi], em = e[hi - 1];
    const double fm = (hi - 1 > lo) ? e[hi - 2] : 0.0;
    const double t11 = dm * dm + fm * fm, t12 = dm * em, t22 = dn * dn + em * em;
    const double half = 0.5 * (t11 - t22);
    const double root = norm2(half, t12);
    const double mu = t22 - t12 * t12 / (half + (half >= 0.0 ? root : -root) + (root == 0.0 ? 1.0 : 0.0));
    // One chase step at column c of a sweep whose bulge state is (y, z).
    auto chase = [&](int c, double &y, double &z) __attribute__((always_inline)) {
      // right rotation on columns (c, c+1) zeroing z against y
      const Rot h = make_rot(y, z);
      if (c > lo) e[c - 1] = h.r;
      {
        const double dc = d[c], ec = e[c], dn1 = d[c + 1];
        d[c] = h.c * dc + h.s * ec;
        e[c] = -h.s * dc + h.c * ec;
        z = h.s * dn1;           // bulge B[c+1][c]
        d[c + 1] = h.c * dn1;
      }
      acc.right(c, c + 1, h.c, h.s);
      // left rotation on rows (c, c+1) zeroing the bulge against d[c]
      const Rot g = make_rot(d[c], z);
      d[c] = g.r;
      {
        const double ec = e[c], dn1 = d[c + 1];
        e[c] = g.c * ec + g.s * dn1;
        d[c + 1] = -g.s * ec + g.c * dn1;
        if (c + 1 < hi) {
          const double en = e[c + 1];
          z = g.s * en;          // bulge B[c][c+2]
          e[c + 1] = g.c * en;
        }
      }
      acc.left(c, c + 1, g.c, g.s);
      y = e[c];
    };
    if (hi - lo < kPairMin) {
      double y = d[lo] * d[lo] - mu;
      double z = d[lo] * e[lo];
      for (int c = lo; c < hi; ++c) chase(c, y, z);
      continue;
    }
    // Two sweeps, with the shift above and with the other eigenvalue of the
    // trailing 2 x 2 of B^T B, the second kPairLag columns behind the first:
    // they touch disjoint entries, so this is the two sweeps one after the
    // other (every rotation that shares a row or column with a later one of
    // the other sweep comes first), but the two dependency chains overlap.
    const double mu2 = std::max(t11 + t22 - mu, 0.0);
    double ya = d[lo] * d[lo] - mu, za = d[lo] * e[lo];
    double yb = 0.0, zb = 0.0;
    for (int c = lo; c < hi + kPairLag; ++c) {
      if (c < hi) chase(c, ya, za);
      const int cb = c - kPairLag;
      if (cb == lo) {
        yb = d[lo] * d[lo] - mu2;
        zb = d[lo] * e[lo];
      }
      if (cb >= lo) chase(cb, yb, zb);
    }
  }

  // signs and order
  std::vector<signed char> sg(k, 1);
  for (int i = 0; i < k; ++i)
    if (d[i] < 0.0) {
      d[i] = -d[i];
      sg[i] = -1;
    }
  std::vector<int> ord(k);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
  std::vector<double> pl(k);
  for (int i = 0; i < k; ++i) {
    out.sigma[i] = d[ord[i]];
    pl[i] = out.p_last[ord[i]];
    out.src[i] = ord[i];
    out.sgn[i] = sg[ord[i]];
  }
  out.p_last.swap(pl);
  return true;
}

__attribute__((target("avx2,fma"))) bool svd_avx2(const std::vector<double> &d, const std::vector<double> &e,
                                                   BidiagSVD &out) {
  return svd_core(d, e, out);
}

bool svd_base(const std::vector<double> &d, const std::vector<double> &e, BidiagSVD &out) {
  return svd_core(d, e, out);
}

constexpr int kVecChunk = 8;    // vectors per block: a k x 8 block stays in L1
constexpr int kVecThreads = 8;  // threads for a large log
constexpr double kVecThreadWork = 4e6;  // rotations x vectors above which threads pay

// The logged rotations applied in reverse order to a k x W row-major block:
// H on rows (a, b) maps (v_a, v_b) to (c v_a - s v_b, s v_a + c v_b).
template <int W>
__attribute__((always_inline)) inline void apply_log_reverse_core(double *V, const BidiagRot *rots, size_t nrot) {
  // A sweep's rotations act on (c, c+1) for increasing c, so in reverse
  // order each one shares its row a with the next one's row b: that row is
  // carried in registers instead of making a round trip through memory.
  double cr[W];
  int crow = -1;
  for (int i = 0; i < W; ++i) cr[i] = 0.0;
  for (size_t t = nrot; t-- > 0;) {
    const BidiagRot h = rots[t];
    double *va = V + (size_t)h.a * W, *vb = V + (size_t)h.b * W;
    double x[W], y[W];
    if (h.b == crow) {
      for (int i = 0; i < W; ++i) y[i] = cr[i];
    } else {
      for (int i = 0; i < W; ++i) y[i] = vb[i];
    }
    for (int i = 0; i < W; ++i) x[i] = va[i];
    for (int i = 0; i < W; ++i) {
      // x's products first: the carried y then enters one multiply-add
      const double cx = h.c * x[i], sx = h.s * x[i];
      const double na = cx - h.s * y[i];
      const double nb = sx + h.c * y[i];
      va[i] = na;
      vb[i] = nb;
      cr[i] = na;
    }
    crow = h.a;
  }
}

__attribute__((target("avx2,fma"))) void apply_log_reverse_avx2(double *V, const BidiagRot *rots, size_t nrot) {
  apply_log_reverse_core<kVecChunk>(V, rots, nrot);
}

void apply_log_reverse_base(double *V, const BidiagRot *rots, size_t nrot) {
  apply_log_reverse_core<kVecChunk>(V, rots, nrot);
}

}  // namespace

bool bidiag_svd(const std::vector<double> &d, const std::vector<double> &e, BidiagSVD &out) {
  return have_avx2_fma() ? svd_avx2(d, e, out) : svd_base(d, e, out);
}

void bidiag_vectors(const std::vector<double> &d_in, const std::vector<double> &e_in, int nvec,
                    BidiagSVD &out) {
  const int k = (int)d_in.size();
  nvec = std::max(0, std::min(nvec, k));
  out.nvec = nvec;
  out.Q.assign((size_t)k * nvec, 0.0);
  out.P.assign((size_t)k * nvec, 0.0);
  if (nvec == 0) return;
  // Q = H_1 H_2 ... H_n (Q <- Q H per rotation, from the identity), so
  // column j of Q is H_1 (H_2 (... (H_n e_j))): the rotations applied in
  // reverse order to unit vectors.  The vectors are independent, so they are
  // taken kVecChunk at a time: a block of k x kVecChunk stays in the L1
  // cache while the whole log streams past it, and a large log spreads the
  // blocks over threads.
  const int nchunk = (nvec + kVecChunk - 1) / kVecChunk;
  std::vector<double> V((size_t)nchunk * k * kVecChunk, 0.0);  // [block][row][kVecChunk]
  for (int i = 0; i < nvec; ++i)
    V[((size_t)(i / kVecChunk) * k + out.src[i]) * kVecChunk + i % kVecChunk] = 1.0;
  const BidiagRot *rots = out.rots.data();
  const size_t nrot = out.rots.size();
  const bool avx2 = have_avx2_fma();
  auto run = [&](int c0, int c1) {
    for (int c = c0; c < c1; ++c) {
      double *blk = V.data() + (size_t)c * k * kVecChunk;
      if (avx2)
        apply_log_reverse_avx2(blk, rots, nrot);
      else
        apply_log_reverse_base(blk, rots, nrot);
    }
  };
  const int nthr = ((double)nrot * nvec > kVecThreadWork) ? std::min(nchunk, kVecThreads) : 1;
  if (nthr <= 1) {
    run(0, nchunk);
  } else {
    const int per = (nchunk + nthr - 1) / nthr;
    std::vector<std::thread> th;
    for (int c0 = per; c0 < nchunk; c0 += per) th.emplace_back(run, c0, std::min(nchunk, c0 + per));
    run(0, std::min(nchunk, per));
    for (auto &t : th) t.join();
  }
  for (int i = 0; i < nvec; ++i) {
    const double sg = out.sgn[i];
    double *q = out.Q.data() + (size_t)i * k;
    const double *v = V.data() + (size_t)(i / kVecChunk) * k * kVecChunk + i % kVecChunk;
    for (int j = 0; j < k; ++j) q[j] = sg * v[(size_t)j * kVecChunk];
  }
  // left vectors from the right ones: B q_i = sigma_i p_i with the input B
  // (upper bidiagonal: (B q)_j = d_j q_j + e_j q_{j+1}); accurate to about
  // eps sigma_1 / sigma_i, ample for the values above tau that are used.
  // A zero singular value leaves a zero column.
  for (int i = 0; i < nvec; ++i) {
    const double s = out.sigma[i];
    if (!(s > 0.0)) continue;
    const double *q = out.Q.data() + (size_t)i * k;
    double *pc = out.P.data() + (size_t)i * k;
    double nrm2 = 0.0;
    for (int j = 0; j < k; ++j) {
      const double v = d_in[j] * q[j] + (j + 1 < k ? e_in[j] * q[j + 1] : 0.0);
      pc[j] = v;
      nrm2 += v * v;
    }
    const double inv = 1.0 / std::sqrt(nrm2);
    for (int j = 0; j < k; ++j) pc[j] *= inv;
  }
}

bool bidiag_svd(const std::vector<double> &d, const std::vector<double> &e, bool vectors, BidiagSVD &out) {
  if (!bidiag_svd(d, e, out)) return false;
  if (vectors) bidiag_vectors(d, e, (int)d.size(), out);
  return true;
}

}  // namespace svt
