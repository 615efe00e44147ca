// bank.hip -- template-bank placement at a set mismatch (host only).
//
// The bank of the per-chunk loop is a set of (m1, m2) points placed so that
// no point of the mass range loses more than a set fraction of SNR to its
// nearest template.  Coordinates are the chirp times (tau_0, tau_3) at
// f_0 = f_low; the metric is Owen's (PRD 53, 6749 (1996)): the match of two
// nearby chirps, maximised over phase and time, is 1 - gamma_ab dtau^a dtau^b
// with gamma half the covariance, under the weight f^{-7/3}/S on the band,
// of the phase derivatives along tau_a after projecting out 2 pi f.
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "ci_impl.h"

namespace {

constexpr double kTSun = 4.925490947641267e-6;  // G M_sun / c^3, seconds
constexpr double kPi = 3.14159265358979323846;

struct Band {
  int64_t kl, kh;
};

// Search band of (M, eta) on the grid: [ceil(f_low T), min(floor(f_isco T), n/2 - 1)].
Band band_of(double M, int64_t n, double fs, double f_low) {
  const double T = (double)n / fs;
  const double f_isco = 1.0 / (6.0 * sqrt(6.0) * kPi * M);
  Band b;
  b.kl = (int64_t)ceil(f_low * T);
  const double kh = floor(f_isco * T);
  b.kh = kh < (double)(n / 2 - 1) ? (int64_t)kh : n / 2 - 1;
  return b;
}

// 2PN stationary phase Psi(f) (t_c = phi_c = 0, radians) from (M, eta).
double psi2pn(double f, double M, double eta) {
  const double v = cbrt(kPi * M * f);
  const double v2 = v * v;
  const double pn = 1.0 + (3715.0 / 756.0 + 55.0 * eta / 9.0) * v2 - 16.0 * kPi * v2 * v +
                    (15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta * eta / 72.0) *
                        v2 * v2;
  return -0.25 * kPi + 3.0 / (128.0 * eta * v2 * v2 * v) * pn;
}

void chirp_times(double m1, double m2, double f0, double* t0, double* t3) {
  const double M = (m1 + m2) * kTSun;
  const double eta = m1 * m2 / ((m1 + m2) * (m1 + m2));
  const double x = kPi * M * f0;
  *t0 = 5.0 / (256.0 * kPi * f0 * eta) * pow(x, -5.0 / 3.0);
  *t3 = 1.0 / (8.0 * f0 * eta) * pow(x, -2.0 / 3.0);
}

// (M seconds, eta) from chirp times (eta may exceed 1/4 off the physical
// region).
void m_eta(double t0, double t3, double f0, double* M, double* eta) {
  const double x = 5.0 * t3 / (32.0 * kPi * t0);  // pi M f0
  *M = x / (kPi * f0);
  *eta = 1.0 / (8.0 * f0 * t3) * pow(x, -2.0 / 3.0);
}

// gamma = {g00, g03, g33} at (m1, m2) on its own band; false for an empty band.
bool metric_at(const double* psd, int64_t n, double fs, double f_low, double m1, double m2,
               double* g) {
  const double M = (m1 + m2) * kTSun;
  const Band b = band_of(M, n, fs, f_low);
  if (b.kh < b.kl) return false;
  double t[2];
  chirp_times(m1, m2, f_low, &t[0], &t[1]);
  // phase derivatives along tau_0 and tau_3 by central differences
  double Mp[2], ep[2], Mm[2], em[2], h[2];
  for (int a = 0; a < 2; ++a) {
    h[a] = 1e-6 * t[a];
    double tp[2] = {t[0], t[1]}, tm[2] = {t[0], t[1]};
    tp[a] += h[a];
    tm[a] -= h[a];
    m_eta(tp[0], tp[1], f_low, &Mp[a], &ep[a]);
    m_eta(tm[0], tm[1], f_low, &Mm[a], &em[a]);
  }
  const double df = fs / (double)n;
  double sw = 0.0, s[3] = {0, 0, 0}, ss[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int64_t k = b.kl; k <= b.kh; ++k) {
    const double f = (double)k * df;
    const double w = pow(f, -7.0 / 3.0) / psd[k];
    double p[3];
    p[0] = 2.0 * kPi * f;
    for (int a = 0; a < 2; ++a)
      p[1 + a] = (psi2pn(f, Mp[a], ep[a]) - psi2pn(f, Mm[a], em[a])) / (2.0 * h[a]);
    sw += w;
    for (int i = 0; i < 3; ++i) {
      s[i] += w * p[i];
      for (int j = 0; j < 3; ++j) ss[i][j] += w * p[i] * p[j];
    }
  }
  double C[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i][j] = ss[i][j] / sw - (s[i] / sw) * (s[j] / sw);
  g[0] = 0.5 * (C[1][1] - C[1][0] * C[1][0] / C[0][0]);
  g[1] = 0.5 * (C[1][2] - C[1][0] * C[2][0] / C[0][0]);
  g[2] = 0.5 * (C[2][2] - C[2][0] * C[2][0] / C[0][0]);
  return true;
}

struct P2 {
  double x, y;
};

// Runs f(i) for every i in [0, n) on up to 16 host threads. Each i writes
// only its own slot, so what the caller assembles afterwards does not depend
// on the number of threads; a thread that cannot be started leaves its share
// to the others.
template <class F>
void parallel_for(int64_t n, const F& f) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int64_t nt = std::min<int64_t>(n, hw);
  std::atomic<int64_t> next{0};
  const auto run = [&] {
    for (int64_t i; (i = next.fetch_add(1, std::memory_order_relaxed)) < n;) f(i);
  };
  std::vector<std::thread> th;
  for (int64_t t = 1; t < nt; ++t) {
    try {
      th.emplace_back(run);
    } catch (...) {
      break;
    }
  }
  run();
  for (std::thread& t : th) t.join();
}

// Closest point to p on segment [a, b].
P2 closest_on_segment(P2 p, P2 a, P2 b) {
  const double dx = b.x - a.x, dy = b.y - a.y;
  const double l2 = dx * dx + dy * dy;
  double t = l2 > 0 ? ((p.x - a.x) * dx + (p.y - a.y) * dy) / l2 : 0.0;
  t = t < 0 ? 0 : (t > 1 ? 1 : t);
  return P2{a.x + t * dx, a.y + t * dy};
}

// The part of a polygon with a <= x <= b (Sutherland-Hodgman against the
// two half-planes).
std::vector<P2> clip_half(const std::vector<P2>& in, double c, bool keep_ge) {
  std::vector<P2> out;
  if (in.empty()) return out;
  auto ok = [&](const P2& p) { return keep_ge ? p.x >= c : p.x <= c; };
  for (size_t i = 0; i < in.size(); ++i) {
    const P2 a = in[i], b = in[(i + 1) % in.size()];
    const bool ia = ok(a), ib = ok(b);
    if (ia) out.push_back(a);
    if (ia != ib) {
      const double t = (c - a.x) / (b.x - a.x);
      out.push_back(P2{c, a.y + t * (b.y - a.y)});
    }
  }
  return out;
}

std::vector<P2> clip_slab(const std::vector<P2>& poly, double a, double b) {
  return clip_half(clip_half(poly, a, true), b, false);
}

bool inside(const std::vector<P2>& poly, P2 p) {
  bool in = false;
  for (size_t i = 0, j = poly.size() - 1; i < poly.size(); j = i++) {
    const P2 a = poly[i], b = poly[j];
    if ((a.y > p.y) != (b.y > p.y) && p.x < (b.x - a.x) * (p.y - a.y) / (b.y - a.y) + a.x)
      in = !in;
  }
  return in;
}

// Bounding metric of a set of metrics g_i = {g00, g03, g33}: G = s S with
// det S = 1 and s the smallest factor for which G dominates every g_i (its
// unit ellipse lies inside each of theirs), minimised over the orientation
// and aspect of S by a compass search started from the shape of g_start.
// With S^-1 = [[p, q], [q, r]] the largest eigenvalue of S^-1 g is
// t/2 + sqrt(t^2/4 - det g), t = p g00 + 2 q g03 + r g33.
struct Shape {
  double th, la;  // orientation, log square root of the aspect
};

double bound_factor(const std::vector<const double*>& gs, Shape sh) {
  const double c = cos(sh.th), s = sin(sh.th), a = exp(-sh.la), b = exp(sh.la);
  const double p = a * c * c + b * s * s, q = (a - b) * c * s, r = a * s * s + b * c * c;
  double need = 0.0;
  for (const double* g : gs) {
    const double t = p * g[0] + 2.0 * q * g[1] + r * g[2];
    const double d = g[0] * g[2] - g[1] * g[1];
    need = std::max(need, 0.5 * t + sqrt(std::max(0.0, 0.25 * t * t - d)));
  }
  return need;
}

void bounding_metric(const std::vector<const double*>& gs, const double* g_start, double* G) {
  // shape of g_start: eigenvalues e0 >= e1 at angle th of the first
  const double tr = g_start[0] + g_start[2];
  const double dd = sqrt(0.25 * (g_start[0] - g_start[2]) * (g_start[0] - g_start[2]) +
                         g_start[1] * g_start[1]);
  const double e0 = 0.5 * tr + dd, e1 = 0.5 * tr - dd;
  Shape best{0.5 * atan2(2.0 * g_start[1], g_start[0] - g_start[2]), 0.5 * log(e0 / e1)};
  double fb = bound_factor(gs, best);
  double st_th = 0.1, st_la = 0.25;
  while (st_th > 1e-6 || st_la > 1e-6) {
    bool moved = false;
    const Shape trial[4] = {{best.th + st_th, best.la}, {best.th - st_th, best.la},
                            {best.th, best.la + st_la}, {best.th, best.la - st_la}};
    for (const Shape& t : trial) {
      const double f = bound_factor(gs, t);
      if (f < fb) {
        fb = f;
        best = t;
        moved = true;
      }
    }
    if (!moved) {
      st_th *= 0.5;
      st_la *= 0.5;
    }
  }
  const double c = cos(best.th), s = sin(best.th), a = exp(best.la), b = exp(-best.la);
  G[0] = fb * (a * c * c + b * s * s);
  G[1] = fb * (a - b) * c * s;
  G[2] = fb * (a * s * s + b * c * c);
}

}  // namespace

extern "C" {

int ci_bank_metric(const double* psd_host, int64_t n, double fs, double f_low, double m1,
                   double m2, double* gamma_out) {
  if (!psd_host || !gamma_out) return ci::report_error(CI_EINVAL, "null psd or output");
  if (n < 16 || (n & (n - 1)) != 0 || !(fs > 0) || !(f_low > 0))
    return ci::report_error(CI_EINVAL, "bad grid");
  if (!(m1 > 0) || !(m2 > 0) || !isfinite(m1) || !isfinite(m2))
    return ci::report_error(CI_EINVAL, "masses must be positive");
  if (!metric_at(psd_host, n, fs, f_low, std::max(m1, m2), std::min(m1, m2), gamma_out))
    return ci::report_error(CI_EINVAL, "empty band");
  return CI_OK;
}

int ci_make_bank_lattice(const ci_lattice_spec* spec, const double* psd_host, int64_t n,
                         double fs, double f_low, ci_template* out_host, int64_t cap,
                         int64_t* count) {
  if (!spec || !psd_host || !count) return ci::report_error(CI_EINVAL, "null argument");
  if (cap < 0 || (cap > 0 && !out_host)) return ci::report_error(CI_EINVAL, "bad output");
  const double lo = spec->m_min, hi = spec->m_max, mm = 1.0 - spec->min_match;
  if (!(lo > 0) || !(hi > lo) || !isfinite(hi)) return ci::report_error(CI_EINVAL, "bad mass range");
  if (!(spec->min_match > 0.5) || !(spec->min_match < 1.0))
    return ci::report_error(CI_EINVAL, "min_match outside (0.5, 1)");
  if (n < 16 || (n & (n - 1)) != 0 || !(fs > 0) || !(f_low > 0))
    return ci::report_error(CI_EINVAL, "bad grid");
  {
    const Band b = band_of(2.0 * hi * kTSun, n, fs, f_low);
    if (b.kh < b.kl) return ci::report_error(CI_EINVAL, "the heaviest templates have no band");
  }
  // boundary of the range in (tau_0, tau_3): m2 = lo (m1 up), m1 = hi (m2
  // up), m1 = m2 (down)
  const int S = 512;
  std::vector<P2> region;
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < S; ++i) {
      const double r = pow(hi / lo, (double)i / S);
      double m1, m2;
      if (e == 0) { m1 = lo * r; m2 = lo; }
      else if (e == 1) { m1 = hi; m2 = lo * r; }
      else { m1 = hi / r; m2 = m1; }
      P2 t;
      chirp_times(m1, m2, f_low, &t.x, &t.y);
      region.push_back(t);
    }
  // metric samples on a log grid of (m1 >= m2), computed in parallel and
  // kept in grid order
  struct Sample {
    P2 t;
    double g[3];
  };
  const int G = 24;
  std::vector<P2> grid;
  for (int i = 0; i < G; ++i)
    for (int j = 0; j <= i; ++j)
      grid.push_back(P2{lo * pow(hi / lo, (double)i / (G - 1)), lo * pow(hi / lo, (double)j / (G - 1))});
  std::vector<Sample> all(grid.size());
  std::vector<char> ok(grid.size(), 0);
  parallel_for((int64_t)grid.size(), [&](int64_t q) {
    const double m1 = grid[(size_t)q].x, m2 = grid[(size_t)q].y;
    Sample& sm = all[(size_t)q];
    if (!metric_at(psd_host, n, fs, f_low, m1, m2, sm.g)) return;
    chirp_times(m1, m2, f_low, &sm.t.x, &sm.t.y);
    ok[(size_t)q] = 1;
  });
  std::vector<Sample> samples;
  for (size_t q = 0; q < grid.size(); ++q)
    if (ok[q]) samples.push_back(all[q]);
  if (samples.empty()) return ci::report_error(CI_EINVAL, "no template of the range has a band");
  double t0min = 1e300, t0max = -1e300;
  for (const P2& p : region) {
    t0min = std::min(t0min, p.x);
    t0max = std::max(t0max, p.x);
  }
  // strips of equal width in log tau_0, each with its own bounding metric
  // and lattice, covering its part of the range: 12, or fewer when the
  // range spans less than 10 covering radii per strip along tau_0 (each
  // strip adds edge points, which dominate a narrow range)
  const double R = sqrt(mm), side = sqrt(3.0 * mm), dy = side * sqrt(3.0) / 2.0;
  std::vector<double> g00;
  for (const Sample& sm : samples) g00.push_back(sm.g[0]);
  std::nth_element(g00.begin(), g00.begin() + g00.size() / 2, g00.end());
  const double extent = sqrt(g00[g00.size() / 2]) * (t0max - t0min);
  const int K = (int)std::min(12.0, std::max(1.0, floor(extent / (10.0 * R))));
  // Each strip is set up in turn (polygon, bounding metric, bounds); its
  // lattice rows are then placed in parallel, in blocks whose results are
  // joined in strip and row order.
  struct Strip {
    std::vector<P2> pu;
    double l00, l10, l11, sq, xmin, xmax, ymin, ymax;
    int64_t rows;
  };
  std::vector<Strip> strips;
  double work = 0.0;
  for (int st = 0; st < K; ++st) {
    const double a = t0min * pow(t0max / t0min, (double)st / K);
    const double b = st == K - 1 ? t0max * (1 + 1e-12) : t0min * pow(t0max / t0min, (double)(st + 1) / K);
    std::vector<P2> poly = clip_slab(region, a, b);
    if (poly.size() < 3) continue;
    // metric samples of the strip (the nearest ones when it holds few)
    std::vector<const Sample*> in;
    for (const Sample& sm : samples)
      if (sm.t.x >= a && sm.t.x < b) in.push_back(&sm);
    if (in.size() < 4) {
      std::vector<std::pair<double, const Sample*>> by;
      const double mid = sqrt(a * b);
      for (const Sample& sm : samples) by.push_back({fabs(log(sm.t.x / mid)), &sm});
      std::sort(by.begin(), by.end(),
                [](const std::pair<double, const Sample*>& u, const std::pair<double, const Sample*>& v) {
                  return u.first < v.first;
                });
      in.clear();
      for (size_t q = 0; q < by.size() && q < 6; ++q) in.push_back(by[q].second);
    }
    // the strip's metric: the smallest one that bounds its samples (search
    // started from the sample nearest the strip's middle), gc = L L^T
    const Sample* ref = in[0];
    for (const Sample* sm : in)
      if (fabs(log(sm->t.x / sqrt(a * b))) < fabs(log(ref->t.x / sqrt(a * b)))) ref = sm;
    std::vector<const double*> gs;
    for (const Sample* sm : in) gs.push_back(sm->g);
    double gc[3];
    bounding_metric(gs, ref->g, gc);
    Strip sp;
    sp.l00 = sqrt(gc[0]);
    sp.l10 = gc[1] / sp.l00;
    sp.l11 = sqrt(gc[2] - sp.l10 * sp.l10);
    const double scale = 1.05;
    // u = sqrt(scale) L^T tau: the bounding metric is the identity in u
    sp.sq = sqrt(scale);
    for (const P2& t : poly)
      sp.pu.push_back(P2{sp.sq * (sp.l00 * t.x + sp.l10 * t.y), sp.sq * sp.l11 * t.y});
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (const P2& p : sp.pu) {
      xmin = std::min(xmin, p.x); xmax = std::max(xmax, p.x);
      ymin = std::min(ymin, p.y); ymax = std::max(ymax, p.y);
    }
    sp.xmin = xmin - R; sp.xmax = xmax + R; sp.ymin = ymin - R; sp.ymax = ymax + R;
    work += ((sp.ymax - sp.ymin) / dy + 1) * ((sp.xmax - sp.xmin) / side + 1);
    if (work > 5e7) return ci::report_error(CI_EINVAL, "lattice too large (over 5e7 points)");
    sp.rows = 0;
    while (sp.ymin + sp.rows * dy <= sp.ymax) ++sp.rows;
    strips.push_back(std::move(sp));
  }
  const int64_t kRowBlock = 16;
  struct Block {
    size_t strip;
    int64_t r0, r1;
  };
  std::vector<Block> blocks;
  for (size_t i = 0; i < strips.size(); ++i)
    for (int64_t r = 0; r < strips[i].rows; r += kRowBlock)
      blocks.push_back(Block{i, r, std::min(strips[i].rows, r + kRowBlock)});
  std::vector<std::vector<ci_template>> placed(blocks.size());
  parallel_for((int64_t)blocks.size(), [&](int64_t bi) {
    const Block& bk = blocks[(size_t)bi];
    const Strip& sp = strips[bk.strip];
    const std::vector<P2>& pu = sp.pu;
    std::vector<ci_template>& dst = placed[(size_t)bi];
    for (int64_t r = bk.r0; r < bk.r1; ++r) {
      const double y = sp.ymin + r * dy, x0 = sp.xmin + ((r & 1) ? 0.5 * side : 0.0);
      for (int64_t c = 0; x0 + c * side <= sp.xmax; ++c) {
        P2 p{x0 + c * side, y};
        if (!inside(pu, p)) {
          // within the covering radius of the strip: move onto its boundary
          P2 best{0, 0};
          double bd = 1e300;
          for (size_t q = 0; q < pu.size(); ++q) {
            const P2 e = closest_on_segment(p, pu[q], pu[(q + 1) % pu.size()]);
            const double d = (e.x - p.x) * (e.x - p.x) + (e.y - p.y) * (e.y - p.y);
            if (d < bd) { bd = d; best = e; }
          }
          if (bd > R * R) continue;
          p = best;
        }
        const double t3 = p.y / (sp.sq * sp.l11), t0 = (p.x / sp.sq - sp.l10 * t3) / sp.l00;
        double M, eta;
        m_eta(t0, t3, f_low, &M, &eta);
        if (!(eta > 0)) continue;
        eta = std::min(eta, 0.25);
        const double mt = M / kTSun, d = sqrt(std::max(0.0, 1.0 - 4.0 * eta));
        ci_template tm;
        tm.m1 = std::min(std::max(0.5 * mt * (1.0 + d), lo), hi);
        tm.m2 = std::min(std::max(0.5 * mt * (1.0 - d), lo), tm.m1);
        dst.push_back(tm);
      }
    }
  });
  std::vector<ci_template> out;
  for (const std::vector<ci_template>& v : placed) out.insert(out.end(), v.begin(), v.end());
  *count = (int64_t)out.size();
  const int64_t k = std::min<int64_t>(cap, (int64_t)out.size());
  for (int64_t i = 0; i < k; ++i) out_host[i] = out[(size_t)i];
  return (int64_t)out.size() > cap && cap > 0 ? CI_ETRUNC : CI_OK;
}

}  // extern "C"
