// FP64 reference ("oracle") of the particle-based grain-envelope step.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
// import or call this file or the library built from it; only the tests, the
// smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
// with the HIP implementation: the two agree only on the semantic contract.
//
// The method (Mosbah et al., "A particle-based approach for the prediction of
// grain microstructures in solidification processes", arXiv:2504.12858):
//   * nucleation: pre-drawn sites with a nucleation undercooling each fire when
//     the local undercooling reaches it (Sec. 2.1.1);
//   * growth: tracking particles move along the grain's rotated <100> axes at
//     the tip velocity of the kinetic law, Eq. (1)/(2), evaluated with each
//     particle's own undercooling (Sec. 2.1.2);
//   * branching: a particle that has travelled lambda0 to its target spawns a
//     new pattern of particles there, keeping only the outer directions that
//     grow the grain (Sec. 2.1.2, Fig. 2);
//   * competition: particles of two different grains that meet stop, forming a
//     grain boundary (Sec. 2.1.2);
//   * rendering: a voxel is labelled with the grain owning its nearest lattice
//     site (Voronoi kernel interpolation, Sec. 2.3).
//
// Readings where the paper is silent (each also listed in the design notes):
//   R1 directions d = 0..5 are (+x,-x,+y,-y,+z,-z) of the crystal frame; the
//      grain rotation R maps crystal to world, R from a unit quaternion.
//   R2 a particle carries the lattice site it left (integer, crystal frame,
//      spacing lambda0, origin at the grain centre) and its travel s since.
//   R3 "outer" directions at a reached site S: d' with sign(d') * S[axis(d')]
//      >= 0 (the octant rule), whose target S + step(d') is not yet claimed by
//      the grain.  Same-step competitors for one target: the lowest d' wins
//      (competitors always differ in d').  Overshoot s - lambda0 is carried
//      into the children.  The parent always retires: with no surviving child
//      every outer neighbour of S already belongs to the grain, so S is inside
//      the envelope, and the stored point cloud keeps only envelope points
//      (shell-like cloud, Sec. 2.3).
//   R4 two particles of different grains "meet" when their distance is < rc.
//      Decisions are collected first and applied together (Jacobi).
//   R5 a particle leaving the box [lo, hi) stops.
//   R6 v = 0 for dT <= 0; the field is taken at t_n for every phase of step n.
//   R7 a site fires only if it is liquid: no non-retired particle within rc and
//      no grain claims the site's rounded lattice position.  Sites are taken
//      in index order within a step.
//   R8 an initial envelope of L1 radius r claims the full lattice ball of
//      radius r; its particles move along the axis of largest |offset|.
//
// Precision: FP64 throughout, except the FP32 checker functions, which
// reproduce single-rounded FP32 binning and distance tests.  Build with
// -ffp-contract=off so that no multiply-add is fused.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <unordered_set>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum : int32_t { P_ACTIVE = 0, P_STOPPED = 1, P_RETIRED = 2 };
enum : int32_t { S_DORMANT = 0, S_FIRED = 1 };
enum : uint8_t { C_CLAIMED = 1, C_REACHED = 2 };
enum : int32_t { F_UNIFORM = 0, F_LINEAR = 1, F_GRID = 2, F_ROSENTHAL = 3, F_SOLUTE = 4 };
enum : int32_t { E_OK = 0, E_INVAL = -1, E_CAPACITY = -2, E_NUMERIC = -3, E_CFL = -4 };

struct Params {
  double lo[3], hi[3];
  double lambda0, h, rc;
  double a[2], b[2];
  double theta;
  int32_t branching, box_exit;
  int32_t periodic;  // bit a: axis a is periodic with period hi[a] - lo[a]
};

struct Grain {
  double c[3];
  double R[3][3];  // column k = crystal axis k in world coordinates
};

struct Particle {
  int32_t g;
  int32_t site[3];
  int32_t dir;
  double s;
  double x[3];
  int32_t state;
};

struct NucSite {
  double y[3];
  double dTn;
  double q[4];
  int32_t state;
};

struct Field {
  int32_t kind = F_UNIFORM;
  double dT = 0, dT0 = 0, grad[3] = {0, 0, 0}, rate = 0;
  int32_t n[3] = {0, 0, 0};
  double o[3] = {0, 0, 0}, sp[3] = {0, 0, 0};
  std::vector<double> data;  // node values, index (k*ny + j)*nx + i
  // SOLUTE: node temperature and solute concentration, liquidus
  // T_L(w) = liq_T + liq_m w (Sec. 3.4: undercooling taken with respect to
  // the local solute concentration)
  std::vector<double> Tn, wn;
  double liq_T = 0, liq_m = 0;
  double q = 0, U = 0, alpha = 0, x_start = 0, x_end = 0, ys = 0, zs = 0, r_min = 0,
         dT_min = -1000;
  double sampled_t = NAN;  // time at which a Rosenthal grid was last sampled
};

struct Stats {
  int64_t advanced = 0, exited = 0, spawners = 0, children = 0, contained = 0,
          nucleated = 0;
  int64_t melted = 0, removed = 0, reactivated = 0, grains_melted = 0;
  double max_step = 0;
};

using ClaimMap = std::unordered_map<uint64_t, uint8_t>;

struct Oracle {
  Params p{};
  std::vector<Grain> grains;
  std::vector<ClaimMap> claims;
  std::vector<Particle> parts;
  std::vector<NucSite> sites;
  Field f;
  double t = 0;
  int64_t step = 0;
  int32_t err = E_OK;
  Stats last;
  bool melting = false;
  std::vector<int32_t> grain_site;  // nucleation site of each grain, -1 for initial grains
};

inline int axis_of(int d) { return d >> 1; }
inline int sign_of(int d) { return (d & 1) ? -1 : 1; }

inline uint64_t site_key(int32_t x, int32_t y, int32_t z) {
  const uint64_t off = 1u << 20;
  return ((uint64_t)(x + off) << 42) | ((uint64_t)(y + off) << 21) | (uint64_t)(z + off);
}

void rotation_from_quat(const double q_in[4], double R[3][3]) {
  double w = q_in[0], x = q_in[1], y = q_in[2], z = q_in[3];
  double n = std::sqrt(w * w + x * x + y * y + z * z);
  w /= n; x /= n; y /= n; z /= n;
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

// World position of lattice site `site` plus travel s along direction d.
void lattice_position(const Params& p, const Grain& g, const int32_t site[3], int d, double s,
                      double out[3]) {
  double loc[3] = {p.lambda0 * site[0], p.lambda0 * site[1], p.lambda0 * site[2]};
  loc[axis_of(d)] += sign_of(d) * s;
  for (int i = 0; i < 3; ++i)
    out[i] = g.c[i] + g.R[i][0] * loc[0] + g.R[i][1] * loc[1] + g.R[i][2] * loc[2];
}

// Growth direction R e_d in world coordinates.
void direction(const Grain& g, int d, double u[3]) {
  int a = axis_of(d);
  double sg = sign_of(d);
  for (int i = 0; i < 3; ++i) u[i] = sg * g.R[i][a];
}

// Kinetic law, Eq. (2): v = a1 dT^b1 + a2 dT^b2 for dT > 0, else 0.
double velocity(const Params& p, double dT) {
  if (!(dT > 0)) return 0.0;
  return p.a[0] * std::pow(dT, p.b[0]) + p.a[1] * std::pow(dT, p.b[1]);
}

// dv/d(dT) for the adjoint.
double velocity_slope(const Params& p, double dT) {
  if (!(dT > 0)) return 0.0;
  return p.a[0] * p.b[0] * std::pow(dT, p.b[0] - 1) + p.a[1] * p.b[1] * std::pow(dT, p.b[1] - 1);
}

// ---------------------------------------------------------------- field ----

double rosenthal_node(const Field& f, double X, double Y, double Z, double t) {
  // Background: linear undercooling.  Source: Rosenthal moving point source
  // T - T_bg = q/(2 pi r) exp(-U (xi + r) / (2 alpha)), xi along the travel
  // direction, rastering back and forth between x_start and x_end.
  double L = f.x_end - f.x_start;
  double travel = f.U * t;
  double phase = std::fmod(travel, 2 * L);
  double xs, sgn;
  if (phase < L) { xs = f.x_start + phase; sgn = 1; }
  else { xs = f.x_start + 2 * L - phase; sgn = -1; }
  double xi = sgn * (X - xs);
  double dy = Y - f.ys, dz = Z - f.zs;
  double r = std::sqrt(xi * xi + dy * dy + dz * dz);
  if (r < f.r_min) r = f.r_min;
  double rise = f.q / (2 * M_PI * r) * std::exp(-f.U * (xi + r) / (2 * f.alpha));
  double dT = f.dT0 + f.grad[0] * X + f.grad[1] * Y + f.grad[2] * Z + f.rate * t - rise;
  if (dT < f.dT_min) dT = f.dT_min;
  return dT;
}

void sample_rosenthal(Field& f, double t) {
  if (f.sampled_t == t) return;
  const int nx = f.n[0], ny = f.n[1], nz = f.n[2];
  f.data.resize((size_t)nx * ny * nz);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        f.data[((size_t)k * ny + j) * nx + i] =
            rosenthal_node(f, f.o[0] + i * f.sp[0], f.o[1] + j * f.sp[1], f.o[2] + k * f.sp[2], t);
  f.sampled_t = t;
}

// Trilinear interpolation of node values `data` on the field's node-centred
// grid; cell index clamped to [0, n-2], fraction clamped to [0, 1].
// Optionally returns the gradient of the interpolant (zero along an axis
// whose fraction was clamped).
double trilinear(const Field& f, const std::vector<double>& data, const double x[3],
                 double grad[3]) {
  int i0[3];
  double fr[3];
  bool clamped[3];
  for (int a = 0; a < 3; ++a) {
    double u = (x[a] - f.o[a]) / f.sp[a];
    double fl = std::floor(u);
    int i = (int)fl;
    if (fl < 0) i = 0;
    if (fl > f.n[a] - 2) i = f.n[a] - 2;
    double w = u - i;
    clamped[a] = false;
    if (w < 0) { w = 0; clamped[a] = true; }
    if (w > 1) { w = 1; clamped[a] = true; }
    i0[a] = i;
    fr[a] = w;
  }
  const int nx = f.n[0], ny = f.n[1];
  auto at = [&](int di, int dj, int dk) {
    return data[((size_t)(i0[2] + dk) * ny + (i0[1] + dj)) * nx + (i0[0] + di)];
  };
  double v = 0;
  double g[3] = {0, 0, 0};
  for (int dk = 0; dk < 2; ++dk)
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) {
        double wx = di ? fr[0] : 1 - fr[0];
        double wy = dj ? fr[1] : 1 - fr[1];
        double wz = dk ? fr[2] : 1 - fr[2];
        double val = at(di, dj, dk);
        v += wx * wy * wz * val;
        g[0] += (di ? 1.0 : -1.0) * wy * wz * val;
        g[1] += wx * (dj ? 1.0 : -1.0) * wz * val;
        g[2] += wx * wy * (dk ? 1.0 : -1.0) * val;
      }
  if (grad) {
    for (int a = 0; a < 3; ++a) grad[a] = clamped[a] ? 0.0 : g[a] / f.sp[a];
  }
  return v;
}

// Undercooling field value (without the offset theta) at x and time t.
double field_value(const Field& f, const double x[3], double t, double grad[3] = nullptr) {
  switch (f.kind) {
    case F_UNIFORM:
      if (grad) grad[0] = grad[1] = grad[2] = 0;
      return f.dT;
    case F_LINEAR:
      if (grad) for (int a = 0; a < 3; ++a) grad[a] = f.grad[a];
      return f.dT0 + f.grad[0] * x[0] + f.grad[1] * x[1] + f.grad[2] * x[2] + f.rate * t;
    case F_GRID:
    case F_ROSENTHAL:
      return trilinear(f, f.data, x, grad);
    case F_SOLUTE: {
      // Liquidus of the interpolated concentration minus the interpolated
      // temperature.
      double gT[3], gw[3];
      const double T = trilinear(f, f.Tn, x, grad ? gT : nullptr);
      const double w = trilinear(f, f.wn, x, grad ? gw : nullptr);
      if (grad)
        for (int a = 0; a < 3; ++a) grad[a] = f.liq_m * gw[a] - gT[a];
      return (f.liq_T + f.liq_m * w) - T;
    }
  }
  return NAN;
}

// ---------------------------------------------------------------- claims ---

inline bool claimed(const ClaimMap& m, const int32_t s[3]) {
  return m.find(site_key(s[0], s[1], s[2])) != m.end();
}

inline void add_claim(ClaimMap& m, const int32_t s[3], uint8_t flags) {
  m[site_key(s[0], s[1], s[2])] |= flags;
}

// Rounded lattice position of world point y in grain g (crystal frame).
void lattice_round(const Params& p, const Grain& g, const double y[3], int32_t out[3]) {
  double d[3] = {y[0] - g.c[0], y[1] - g.c[1], y[2] - g.c[2]};
  for (int k = 0; k < 3; ++k) {
    double loc = g.R[0][k] * d[0] + g.R[1][k] * d[1] + g.R[2][k] * d[2];
    out[k] = (int32_t)std::nearbyint(loc / p.lambda0);
  }
}

// ------------------------------------------------ periodic boundaries ----
// Periodic axes (reading R16; Sec. 3.4 applies periodic conditions on the
// faces normal to x and y): the domain repeats with period L = hi - lo.
// Positions stay lattice-anchored and unwrapped; the field, the cell of a
// particle, the deposition cell and the grain map take the position wrapped
// into the box, and distances are taken between nearest periodic images.
inline bool periodic_axis(const Params& p, int a) { return ((p.periodic >> a) & 1) != 0; }

void wrap_pos(const Params& p, const double x[3], double w[3]) {
  for (int a = 0; a < 3; ++a) {
    w[a] = x[a];
    if (!periodic_axis(p, a)) continue;
    const double L = p.hi[a] - p.lo[a];
    w[a] = x[a] - L * std::floor((x[a] - p.lo[a]) / L);
  }
}

// Displacement from b to a between nearest images; returns whether that
// image is not b itself (some periodic shift is non-zero).
bool min_image(const Params& p, const double a[3], const double b[3], double d[3]) {
  bool shifted = false;
  for (int a_ = 0; a_ < 3; ++a_) {
    d[a_] = a[a_] - b[a_];
    if (!periodic_axis(p, a_)) continue;
    const double L = p.hi[a_] - p.lo[a_];
    const double k = std::nearbyint(d[a_] / L);
    d[a_] -= k * L;
    if (k != 0) shifted = true;
  }
  return shifted;
}

// Two particles touch (R4): within rc of each other's nearest image, and of
// different grains or, for one grain, through a periodic image (a grain
// that has grown around the period meets itself).
bool touch(const Params& p, const Particle& a, const Particle& b, double rc2) {
  double d[3];
  const bool shifted = min_image(p, a.x, b.x, d);
  if (a.g == b.g && !shifted) return false;
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rc2;
}

// Cell index along axis a, wrapped on periodic axes (-1 if outside).
inline int32_t stencil_index(const Params& p, const int32_t n[3], int a, int32_t i) {
  if (i >= 0 && i < n[a]) return i;
  if (!periodic_axis(p, a)) return -1;
  return i < 0 ? i + n[a] : i - n[a];
}

// ---------------------------------------------------------------- cells ----

struct CellIndex {
  int32_t n[3];
  std::unordered_map<int64_t, std::vector<int32_t>> cells;
};

void cell_of(const Params& p, const int32_t n[3], const double x_in[3], int32_t c[3]) {
  double x[3];
  wrap_pos(p, x_in, x);
  for (int a = 0; a < 3; ++a) {
    double u = std::floor((x[a] - p.lo[a]) / p.h);
    int64_t i = (int64_t)u;
    if (u < 0) i = 0;
    if (u > n[a] - 1) i = n[a] - 1;
    c[a] = (int32_t)i;
  }
}

inline int64_t cell_key(const int32_t n[3], int32_t i, int32_t j, int32_t k) {
  return ((int64_t)k * n[1] + j) * n[0] + i;
}

// Cells per axis: ceil(L / h); on a periodic axis the period is a whole
// number of cells, L / h rounded (so that the last cell borders the first).
void grid_dims(const Params& p, int32_t n[3]) {
  for (int a = 0; a < 3; ++a) {
    const double r = (p.hi[a] - p.lo[a]) / p.h;
    double m = periodic_axis(p, a) ? std::nearbyint(r) : std::ceil(r);
    n[a] = (int32_t)std::max(1.0, m);
  }
}

// Bins every non-retired particle (stable: ascending vector index).
CellIndex build_cells(const Oracle& o) {
  CellIndex ci;
  grid_dims(o.p, ci.n);
  for (size_t i = 0; i < o.parts.size(); ++i) {
    const Particle& q = o.parts[i];
    if (q.state == P_RETIRED) continue;
    int32_t c[3];
    cell_of(o.p, ci.n, q.x, c);
    ci.cells[cell_key(ci.n, c[0], c[1], c[2])].push_back((int32_t)i);
  }
  return ci;
}

inline double dist2(const double a[3], const double b[3]) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return dx * dx + dy * dy + dz * dz;
}

// Containment decisions (R4) through the 27-cell stencil of the cell index.
void contain_decisions_cells(const Oracle& o, std::vector<uint8_t>& stop) {
  CellIndex ci = build_cells(o);
  const double rc2 = o.p.rc * o.p.rc;
  stop.assign(o.parts.size(), 0);
  const int64_t np = (int64_t)o.parts.size();
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < np; ++i) {
    const Particle& a = o.parts[i];
    if (a.state != P_ACTIVE) continue;
    int32_t c[3];
    cell_of(o.p, ci.n, a.x, c);
    bool hit = false;
    for (int dk = -1; dk <= 1 && !hit; ++dk)
      for (int dj = -1; dj <= 1 && !hit; ++dj)
        for (int di = -1; di <= 1 && !hit; ++di) {
          int32_t ii = stencil_index(o.p, ci.n, 0, c[0] + di);
          int32_t jj = stencil_index(o.p, ci.n, 1, c[1] + dj);
          int32_t kk = stencil_index(o.p, ci.n, 2, c[2] + dk);
          if (ii < 0 || jj < 0 || kk < 0) continue;
          auto it = ci.cells.find(cell_key(ci.n, ii, jj, kk));
          if (it == ci.cells.end()) continue;
          for (int32_t j : it->second)
            if (touch(o.p, a, o.parts[j], rc2)) { hit = true; break; }
        }
    stop[i] = hit ? 1 : 0;
  }
}

// Same decisions by brute force over all pairs (used to pin the cell index).
void contain_decisions_brute(const Oracle& o, std::vector<uint8_t>& stop) {
  const double rc2 = o.p.rc * o.p.rc;
  stop.assign(o.parts.size(), 0);
  const int64_t np = (int64_t)o.parts.size();
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < np; ++i) {
    const Particle& a = o.parts[i];
    if (a.state != P_ACTIVE) continue;
    // Every periodic image of every other particle (shift k L per periodic
    // axis, |k| <= 2: unwrapped positions lie within one period of the
    // box); a particle's own grain counts through images only.
    int kmax[3];
    for (int c = 0; c < 3; ++c) kmax[c] = ((o.p.periodic >> c) & 1) ? 2 : 0;
    for (int64_t j = 0; j < np && !stop[i]; ++j) {
      const Particle& b = o.parts[j];
      if (b.state == P_RETIRED) continue;
      for (int kz = -kmax[2]; kz <= kmax[2]; ++kz)
        for (int ky = -kmax[1]; ky <= kmax[1]; ++ky)
          for (int kx = -kmax[0]; kx <= kmax[0]; ++kx) {
            if (b.g == a.g && kx == 0 && ky == 0 && kz == 0) continue;
            const double img[3] = {b.x[0] + kx * (o.p.hi[0] - o.p.lo[0]),
                                   b.x[1] + ky * (o.p.hi[1] - o.p.lo[1]),
                                   b.x[2] + kz * (o.p.hi[2] - o.p.lo[2])};
            if (dist2(a.x, img) < rc2) stop[i] = 1;
          }
    }
  }
}

// ---------------------------------------------------------------- phases ---

void phase_advance(Oracle& o, double dt) {
  const Params& p = o.p;
  if (o.f.kind == F_ROSENTHAL) sample_rosenthal(o.f, o.t);
  const int64_t np = (int64_t)o.parts.size();
  int64_t adv = 0;
  double max_step = 0;
  int32_t err = E_OK;
#pragma omp parallel for schedule(static) reduction(+ : adv) reduction(max : max_step)
  for (int64_t i = 0; i < np; ++i) {
    Particle& q = o.parts[i];
    if (q.state != P_ACTIVE) continue;
    const Grain& g = o.grains[q.g];
    double xw[3];
    wrap_pos(p, q.x, xw);
    double dT = field_value(o.f, xw, o.t) - p.theta;
    double v = velocity(p, dT);
    double d = v * dt;
    if (!std::isfinite(d)) {
#pragma omp atomic write
      err = E_NUMERIC;
      continue;
    }
    double u[3];
    direction(g, q.dir, u);
    q.s += d;
    for (int a = 0; a < 3; ++a) q.x[a] += d * u[a];
    adv += 1;
    if (d > max_step) max_step = d;
  }
  o.last.advanced = adv;
  o.last.max_step = max_step;
  if (err != E_OK && o.err == E_OK) o.err = err;
  if (max_step > 0.5 * p.rc && o.err == E_OK) o.err = E_CFL;
}

void phase_box_exit(Oracle& o) {
  const Params& p = o.p;
  int64_t n = 0;
  if (!p.box_exit) { o.last.exited = 0; return; }
  for (Particle& q : o.parts) {
    if (q.state != P_ACTIVE) continue;
    bool inside = true;
    for (int a = 0; a < 3; ++a)
      if (!periodic_axis(p, a) && !(q.x[a] >= p.lo[a] && q.x[a] < p.hi[a])) inside = false;
    if (!inside) { q.state = P_STOPPED; ++n; }
  }
  o.last.exited = n;
}

void phase_branch(Oracle& o) {
  const Params& p = o.p;
  o.last.spawners = 0;
  o.last.children = 0;
  if (!p.branching) return;
  std::vector<int64_t> spawners;
  for (size_t i = 0; i < o.parts.size(); ++i) {
    const Particle& q = o.parts[i];
    if (q.state == P_ACTIVE && q.s >= p.lambda0) spawners.push_back((int64_t)i);
  }
  if (spawners.empty()) return;
  // Reached sites of this step, per grain.
  std::vector<std::unordered_set<uint64_t>> reached_now(o.grains.size());
  std::vector<std::array<int32_t, 3>> S(spawners.size());
  for (size_t k = 0; k < spawners.size(); ++k) {
    const Particle& q = o.parts[spawners[k]];
    if (q.s >= 2 * p.lambda0 && o.err == E_OK) o.err = E_CFL;
    int a = axis_of(q.dir);
    S[k] = {q.site[0], q.site[1], q.site[2]};
    S[k][a] += sign_of(q.dir);
    reached_now[q.g].insert(site_key(S[k][0], S[k][1], S[k][2]));
  }
  // Candidates against the claims held before this step.
  struct Cand { size_t k; int d; int32_t T[3]; };
  std::vector<Cand> cands;
  // Lowest competing direction per (grain, target).
  std::unordered_map<int32_t, std::unordered_map<uint64_t, int>> best_by_grain;
  for (size_t k = 0; k < spawners.size(); ++k) {
    const Particle& q = o.parts[spawners[k]];
    for (int d = 0; d < 6; ++d) {
      int a = axis_of(d);
      if (sign_of(d) * S[k][a] < 0) continue;  // octant rule
      Cand c{k, d, {S[k][0], S[k][1], S[k][2]}};
      c.T[a] += sign_of(d);
      if (claimed(o.claims[q.g], c.T)) continue;
      if (reached_now[q.g].count(site_key(c.T[0], c.T[1], c.T[2]))) continue;
      cands.push_back(c);
      auto& m = best_by_grain[q.g];
      uint64_t tk = site_key(c.T[0], c.T[1], c.T[2]);
      auto it = m.find(tk);
      if (it == m.end() || d < it->second) m[tk] = d;
    }
  }
  // Children of each parent, in (parent order, d') order.
  std::vector<int> nchild(spawners.size(), 0);
  std::vector<Particle> born;
  for (const Cand& c : cands) {
    const Particle& q = o.parts[spawners[c.k]];
    if (best_by_grain[q.g][site_key(c.T[0], c.T[1], c.T[2])] != c.d) continue;
    Particle ch{};
    ch.g = q.g;
    for (int a = 0; a < 3; ++a) ch.site[a] = S[c.k][a];
    ch.dir = c.d;
    ch.s = q.s - p.lambda0;
    lattice_position(p, o.grains[q.g], ch.site, ch.dir, ch.s, ch.x);
    ch.state = P_ACTIVE;
    born.push_back(ch);
    nchild[c.k] += 1;
    add_claim(o.claims[q.g], c.T, C_CLAIMED);
  }
  for (size_t k = 0; k < spawners.size(); ++k) {
    Particle& q = o.parts[spawners[k]];
    add_claim(o.claims[q.g], S[k].data(), C_REACHED);
    q.state = P_RETIRED;
  }
  o.last.spawners = (int64_t)spawners.size();
  o.last.children = (int64_t)born.size();
  o.parts.insert(o.parts.end(), born.begin(), born.end());
}

void phase_contain(Oracle& o) {
  std::vector<uint8_t> stop;
  contain_decisions_cells(o, stop);
  int64_t n = 0;
  for (size_t i = 0; i < o.parts.size(); ++i)
    if (stop[i]) { o.parts[i].state = P_STOPPED; ++n; }
  o.last.contained = n;
}

void add_grain(Oracle& o, const double c[3], const double q[4], int32_t site = -1) {
  Grain g{};
  for (int a = 0; a < 3; ++a) g.c[a] = c[a];
  rotation_from_quat(q, g.R);
  o.grains.push_back(g);
  o.claims.emplace_back();
  o.grain_site.push_back(site);
}

inline void site_of_key(uint64_t key, int32_t s[3]) {
  const uint64_t m21 = (1u << 21) - 1;
  const int32_t off = 1 << 20;
  s[0] = (int32_t)((key >> 42) & m21) - off;
  s[1] = (int32_t)((key >> 21) & m21) - off;
  s[2] = (int32_t)(key & m21) - off;
}

// Melting by walk-back (Sec. 2.1.3; reading R15), with the field at t_n:
//   1. a reached site S whose undercooling is negative, dT(x_S) < 0, melts:
//      it is no longer claimed or reached;
//   2. a particle (active or stopped) whose departure site melted is
//      removed, and an active one's target is no longer claimed;
//   3. walk-back: for each site T melted in this step, the first direction d
//      (0..5) for which S = T - e_d is still a reached site of the grain gives
//      an active particle at S moving towards T (travel 0), and T is claimed
//      as its target (the re-activated points are the solid sites next to
//      the melt, within lambda0 of the dT = 0 iso-surface);
//   4. a grain left without reached sites has melted entirely; its
//      nucleation site, if it has one, is dormant again and may fire anew.
void phase_melt(Oracle& o) {
  const Params& p = o.p;
  if (!o.melting) return;
  if (o.f.kind == F_ROSENTHAL) sample_rosenthal(o.f, o.t);
  std::vector<std::vector<uint64_t>> melted(o.grains.size());
  for (size_t g = 0; g < o.grains.size(); ++g) {
    for (auto& kv : o.claims[g]) {
      if (!(kv.second & C_REACHED)) continue;
      int32_t S[3];
      site_of_key(kv.first, S);
      double x[3], xw[3];
      lattice_position(p, o.grains[g], S, 0, 0.0, x);
      wrap_pos(p, x, xw);
      if (field_value(o.f, xw, o.t) - p.theta < 0) melted[g].push_back(kv.first);
    }
    std::sort(melted[g].begin(), melted[g].end());
    for (uint64_t k : melted[g]) o.claims[g].erase(k);
    o.last.melted += (int64_t)melted[g].size();
  }
  // Particles of melted departure sites.
  for (Particle& q : o.parts) {
    if (q.state == P_RETIRED) continue;
    const auto& mg = melted[q.g];
    if (!std::binary_search(mg.begin(), mg.end(), site_key(q.site[0], q.site[1], q.site[2])))
      continue;
    if (q.state == P_ACTIVE) {
      int32_t T[3] = {q.site[0], q.site[1], q.site[2]};
      T[axis_of(q.dir)] += sign_of(q.dir);
      auto it = o.claims[q.g].find(site_key(T[0], T[1], T[2]));
      if (it != o.claims[q.g].end() && it->second == C_CLAIMED) o.claims[q.g].erase(it);
    }
    q.state = P_RETIRED;
    o.last.removed += 1;
  }
  // Walk-back.
  for (size_t g = 0; g < o.grains.size(); ++g) {
    for (uint64_t k : melted[g]) {
      int32_t T[3];
      site_of_key(k, T);
      for (int d = 0; d < 6; ++d) {
        int32_t S[3] = {T[0], T[1], T[2]};
        S[axis_of(d)] -= sign_of(d);
        auto it = o.claims[g].find(site_key(S[0], S[1], S[2]));
        if (it == o.claims[g].end() || !(it->second & C_REACHED)) continue;
        Particle ch{};
        ch.g = (int32_t)g;
        for (int a = 0; a < 3; ++a) ch.site[a] = S[a];
        ch.dir = d;
        ch.s = 0;
        lattice_position(p, o.grains[g], ch.site, ch.dir, 0.0, ch.x);
        ch.state = P_ACTIVE;
        o.parts.push_back(ch);
        add_claim(o.claims[g], T, C_CLAIMED);
        o.last.reactivated += 1;
        break;
      }
    }
    // A grain without reached sites has melted entirely.
    if (!melted[g].empty()) {
      bool any = false;
      for (auto& kv : o.claims[g])
        if (kv.second & C_REACHED) { any = true; break; }
      if (!any) {
        o.claims[g].clear();
        o.last.grains_melted += 1;
        if (o.grain_site[g] >= 0) o.sites[o.grain_site[g]].state = S_DORMANT;
      }
    }
  }
}

void phase_nucleate(Oracle& o) {
  const Params& p = o.p;
  o.last.nucleated = 0;
  if (o.sites.empty()) return;
  if (o.f.kind == F_ROSENTHAL) sample_rosenthal(o.f, o.t);
  const double rc2 = p.rc * p.rc;
  // Index of every non-retired particle; particles born from sites fired
  // earlier in this step are added to it as they appear.
  CellIndex ci = build_cells(o);
  for (NucSite& st : o.sites) {
    if (st.state != S_DORMANT) continue;
    double yw[3];
    wrap_pos(p, st.y, yw);
    double dT = field_value(o.f, yw, o.t) - p.theta;
    if (!(dT >= st.dTn)) continue;
    // Liquid test, claims part: any grain (including grains nucleated earlier
    // in this step) whose claims contain the rounded lattice position of the
    // site or, on periodic axes, of one of its images.
    bool liquid = true;
    for (size_t g = 0; g < o.grains.size() && liquid; ++g) {
      for (int k = 0; k < 27 && liquid; ++k) {
        const int sh[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
        bool ok = true;
        double y[3];
        for (int a = 0; a < 3; ++a) {
          if (sh[a] != 0 && !periodic_axis(p, a)) ok = false;
          y[a] = st.y[a] + sh[a] * (p.hi[a] - p.lo[a]);
        }
        if (!ok) continue;
        int32_t s[3];
        lattice_round(p, o.grains[g], y, s);
        if (claimed(o.claims[g], s)) liquid = false;
      }
    }
    if (!liquid) continue;
    // Liquid test, particles part: no non-retired particle within rc.
    int32_t c[3];
    cell_of(p, ci.n, st.y, c);
    for (int dk = -1; dk <= 1 && liquid; ++dk)
      for (int dj = -1; dj <= 1 && liquid; ++dj)
        for (int di = -1; di <= 1 && liquid; ++di) {
          int32_t ii = stencil_index(p, ci.n, 0, c[0] + di);
          int32_t jj = stencil_index(p, ci.n, 1, c[1] + dj);
          int32_t kk = stencil_index(p, ci.n, 2, c[2] + dk);
          if (ii < 0 || jj < 0 || kk < 0) continue;
          auto it = ci.cells.find(cell_key(ci.n, ii, jj, kk));
          if (it == ci.cells.end()) continue;
          for (int32_t j : it->second) {
            if (o.parts[j].state == P_RETIRED) continue;
            double d[3];
            min_image(p, o.parts[j].x, st.y, d);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rc2) { liquid = false; break; }
          }
        }
    if (!liquid) continue;
    // Fire: new grain with centre y, 6 particles at the centre.
    st.state = S_FIRED;
    add_grain(o, st.y, st.q, (int32_t)(&st - o.sites.data()));
    int32_t g = (int32_t)o.grains.size() - 1;
    int32_t zero[3] = {0, 0, 0};
    add_claim(o.claims[g], zero, C_CLAIMED | C_REACHED);
    for (int d = 0; d < 6; ++d) {
      Particle ch{};
      ch.g = g;
      ch.dir = d;
      ch.s = 0;
      for (int a = 0; a < 3; ++a) ch.x[a] = st.y[a];
      ch.state = P_ACTIVE;
      o.parts.push_back(ch);
      // Index the new particles so that later sites of this step see them.
      int32_t cc[3];
      cell_of(p, ci.n, ch.x, cc);
      ci.cells[cell_key(ci.n, cc[0], cc[1], cc[2])].push_back((int32_t)o.parts.size() - 1);
    }
    o.last.nucleated += 1;
  }
}

void do_step(Oracle& o, double dt) {
  o.last = Stats{};
  phase_melt(o);
  phase_advance(o, dt);
  phase_box_exit(o);
  phase_branch(o);
  phase_contain(o);
  phase_nucleate(o);
  o.t += dt;
  o.step += 1;
}

}  // namespace

// ======================================================== C interface =====

extern "C" {

struct orc_params {
  double lo[3], hi[3];
  double lambda0, h, rc;
  double a[2], b[2];
  double theta;
  int32_t branching, box_exit;
  int32_t periodic;  // bit a: axis a periodic
};

struct orc_field {
  int32_t kind;
  double dT, dT0, grad[3], rate;
  int32_t n[3];
  double origin[3], spacing[3];
  const float* data;  // GRID node values (host, FP32), (k*ny + j)*nx + i
  double q, U, alpha, x_start, x_end, ys, zs, r_min, dT_min;
  const double* T;    // SOLUTE node temperatures and concentrations (host, FP64)
  const double* w;
  double liq_T, liq_m;
};

void* orc_create(const orc_params* pp) {
  Oracle* o = new Oracle();
  std::memcpy(o->p.lo, pp->lo, sizeof(o->p.lo));
  std::memcpy(o->p.hi, pp->hi, sizeof(o->p.hi));
  o->p.lambda0 = pp->lambda0;
  o->p.h = pp->h;
  o->p.rc = pp->rc;
  o->p.a[0] = pp->a[0]; o->p.a[1] = pp->a[1];
  o->p.b[0] = pp->b[0]; o->p.b[1] = pp->b[1];
  o->p.theta = pp->theta;
  o->p.branching = pp->branching;
  o->p.box_exit = pp->box_exit;
  o->p.periodic = pp->periodic;
  return o;
}

void orc_destroy(void* h) { delete (Oracle*)h; }

int32_t orc_error(void* h) { return ((Oracle*)h)->err; }

void orc_set_theta(void* h, double theta) { ((Oracle*)h)->p.theta = theta; }

void orc_set_kinetics(void* h, const double a[2]) {
  ((Oracle*)h)->p.a[0] = a[0];
  ((Oracle*)h)->p.a[1] = a[1];
}

void orc_set_branching(void* h, int32_t on) { ((Oracle*)h)->p.branching = on; }

void orc_set_melting(void* h, int32_t on) { ((Oracle*)h)->melting = on != 0; }

// Melting counters of the last step: sites melted, particles removed,
// particles re-activated, grains melted entirely.
void orc_melt_stats(void* h, int64_t out[4]) {
  const Stats& s = ((Oracle*)h)->last;
  out[0] = s.melted;
  out[1] = s.removed;
  out[2] = s.reactivated;
  out[3] = s.grains_melted;
}

int32_t orc_set_field(void* h, const orc_field* fs) {
  Oracle& o = *(Oracle*)h;
  Field f;
  f.kind = fs->kind;
  f.dT = fs->dT;
  f.dT0 = fs->dT0;
  for (int a = 0; a < 3; ++a) {
    f.grad[a] = fs->grad[a];
    f.n[a] = fs->n[a];
    f.o[a] = fs->origin[a];
    f.sp[a] = fs->spacing[a];
  }
  f.rate = fs->rate;
  f.q = fs->q; f.U = fs->U; f.alpha = fs->alpha;
  f.x_start = fs->x_start; f.x_end = fs->x_end;
  f.ys = fs->ys; f.zs = fs->zs; f.r_min = fs->r_min; f.dT_min = fs->dT_min;
  if (f.kind == F_GRID || f.kind == F_ROSENTHAL || f.kind == F_SOLUTE) {
    for (int a = 0; a < 3; ++a)
      if (f.n[a] < 2 || !(f.sp[a] > 0)) return E_INVAL;
  }
  const size_t m = (size_t)f.n[0] * f.n[1] * f.n[2];
  if (f.kind == F_GRID) {
    f.data.resize(m);
    for (size_t i = 0; i < m; ++i) f.data[i] = (double)fs->data[i];
  }
  if (f.kind == F_SOLUTE) {
    if (!fs->T || !fs->w) return E_INVAL;
    f.Tn.assign(fs->T, fs->T + m);
    f.wn.assign(fs->w, fs->w + m);
    f.liq_T = fs->liq_T;
    f.liq_m = fs->liq_m;
  }
  o.f = std::move(f);
  return E_OK;
}

// Undercooling field (without theta) and its gradient at n points, time t
// (a ROSENTHAL field is sampled at t first).
void orc_field_value(void* h, int64_t n, const double* x, double t, double* out, double* grad) {
  Oracle& o = *(Oracle*)h;
  if (o.f.kind == F_ROSENTHAL) sample_rosenthal(o.f, t);
  for (int64_t k = 0; k < n; ++k) out[k] = field_value(o.f, x + 3 * k, t, grad ? grad + 3 * k : nullptr);
}

// Appends grains.  shell_r[i] = 0: a 6-particle nucleus at the centre with
// the origin claimed.  shell_r[i] = r > 0: particles on the lattice L1 shell
// of radius r, each moving along its axis of largest |offset| (lowest axis on
// ties), the lattice ball of radius r claimed as reached (R8).  Particles
// outside the box start stopped.
int32_t orc_init_grains(void* h, int32_t n, const double* centre, const double* quat,
                        const int32_t* shell_r) {
  Oracle& o = *(Oracle*)h;
  for (int32_t i = 0; i < n; ++i) {
    add_grain(o, centre + 3 * i, quat + 4 * i);
    int32_t g = (int32_t)o.grains.size() - 1;
    int32_t r = shell_r[i];
    const Grain& G = o.grains[g];
    if (r == 0) {
      int32_t zero[3] = {0, 0, 0};
      add_claim(o.claims[g], zero, C_CLAIMED | C_REACHED);
      for (int d = 0; d < 6; ++d) {
        Particle q{};
        q.g = g; q.dir = d; q.s = 0;
        lattice_position(o.p, G, q.site, d, 0.0, q.x);
        q.state = P_ACTIVE;
        o.parts.push_back(q);
      }
    } else {
      for (int32_t x = -r; x <= r; ++x)
        for (int32_t y = -r; y <= r; ++y)
          for (int32_t z = -r; z <= r; ++z) {
            int32_t l1 = std::abs(x) + std::abs(y) + std::abs(z);
            if (l1 > r) continue;
            int32_t s[3] = {x, y, z};
            add_claim(o.claims[g], s, C_CLAIMED | C_REACHED);
            if (l1 != r) continue;
            int a = 0;
            for (int k = 1; k < 3; ++k)
              if (std::abs(s[k]) > std::abs(s[a])) a = k;
            Particle q{};
            q.g = g;
            for (int k = 0; k < 3; ++k) q.site[k] = s[k];
            q.dir = 2 * a + (s[a] < 0 ? 1 : 0);
            q.s = 0;
            lattice_position(o.p, G, q.site, q.dir, 0.0, q.x);
            bool inside = true;
            for (int k = 0; k < 3; ++k)
              if (!periodic_axis(o.p, k) && !(q.x[k] >= o.p.lo[k] && q.x[k] < o.p.hi[k])) inside = false;
            q.state = (inside || !o.p.box_exit) ? P_ACTIVE : P_STOPPED;
            o.parts.push_back(q);
          }
    }
  }
  return E_OK;
}

int32_t orc_nucleate(void* h, int32_t n, const double* xyz, const double* dTn, const double* quat) {
  Oracle& o = *(Oracle*)h;
  for (int32_t i = 0; i < n; ++i) {
    NucSite s{};
    for (int a = 0; a < 3; ++a) s.y[a] = xyz[3 * i + a];
    s.dTn = dTn[i];
    for (int a = 0; a < 4; ++a) s.q[a] = quat[4 * i + a];
    s.state = S_DORMANT;
    o.sites.push_back(s);
  }
  return E_OK;
}

int32_t orc_step(void* h, double dt, int32_t n_steps) {
  Oracle& o = *(Oracle*)h;
  for (int32_t i = 0; i < n_steps; ++i) {
    do_step(o, dt);
    if (o.err != E_OK) return o.err;
  }
  return o.err;
}

// Individual phases, for tests: 0 advance, 1 box exit, 2 branch, 3 contain,
// 4 nucleate, 5 finish (t += dt, step += 1).
int32_t orc_phase(void* h, int32_t phase, double dt) {
  Oracle& o = *(Oracle*)h;
  switch (phase) {
    case 0: o.last = Stats{}; phase_advance(o, dt); break;
    case 1: phase_box_exit(o); break;
    case 2: phase_branch(o); break;
    case 3: phase_contain(o); break;
    case 4: phase_nucleate(o); break;
    case 5: o.t += dt; o.step += 1; break;
    case 6: phase_melt(o); break;
    default: return E_INVAL;
  }
  return o.err;
}

// Containment decisions on the current state without applying them:
// method 0 = 27-cell stencil, 1 = brute force.
void orc_contain_decisions(void* h, int32_t method, uint8_t* out) {
  Oracle& o = *(Oracle*)h;
  std::vector<uint8_t> stop;
  if (method == 0) contain_decisions_cells(o, stop);
  else contain_decisions_brute(o, stop);
  std::memcpy(out, stop.data(), stop.size());
}

// Counts: 0 particles (all), 1 active, 2 stopped, 3 retired, 4 grains,
// 5 claims, 6 sites, 7 fired sites, 8 reached claims.
int64_t orc_count(void* h, int32_t what) {
  Oracle& o = *(Oracle*)h;
  int64_t n = 0;
  switch (what) {
    case 0: return (int64_t)o.parts.size();
    case 1: for (auto& q : o.parts) n += q.state == P_ACTIVE; return n;
    case 2: for (auto& q : o.parts) n += q.state == P_STOPPED; return n;
    case 3: for (auto& q : o.parts) n += q.state == P_RETIRED; return n;
    case 4: return (int64_t)o.grains.size();
    case 5: for (auto& m : o.claims) n += (int64_t)m.size(); return n;
    case 6: return (int64_t)o.sites.size();
    case 7: for (auto& s : o.sites) n += s.state == S_FIRED; return n;
    case 8: for (auto& m : o.claims) for (auto& kv : m) n += (kv.second & C_REACHED) ? 1 : 0; return n;
  }
  return -1;
}

// Last-step counters: advanced, exited, spawners, children, contained, nucleated.
void orc_last_stats(void* h, int64_t out[6], double* max_step) {
  Oracle& o = *(Oracle*)h;
  out[0] = o.last.advanced; out[1] = o.last.exited; out[2] = o.last.spawners;
  out[3] = o.last.children; out[4] = o.last.contained; out[5] = o.last.nucleated;
  if (max_step) *max_step = o.last.max_step;
}

double orc_time(void* h) { return ((Oracle*)h)->t; }

int32_t orc_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads of the parallel loops from now on (n <= 0: one per processor).
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}

void orc_get_particles(void* h, int32_t* grain, int32_t* site, int32_t* dir, double* s, double* x,
                       int32_t* state) {
  Oracle& o = *(Oracle*)h;
  for (size_t i = 0; i < o.parts.size(); ++i) {
    const Particle& q = o.parts[i];
    grain[i] = q.g;
    for (int a = 0; a < 3; ++a) { site[3 * i + a] = q.site[a]; x[3 * i + a] = q.x[a]; }
    dir[i] = q.dir;
    s[i] = q.s;
    state[i] = q.state;
  }
}

void orc_get_grains(void* h, double* centre, double* R) {
  Oracle& o = *(Oracle*)h;
  for (size_t g = 0; g < o.grains.size(); ++g) {
    for (int a = 0; a < 3; ++a) centre[3 * g + a] = o.grains[g].c[a];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) R[9 * g + 3 * i + j] = o.grains[g].R[i][j];
  }
}

void orc_get_claims(void* h, int32_t* grain, int32_t* site, uint8_t* flags) {
  Oracle& o = *(Oracle*)h;
  size_t k = 0;
  const uint64_t m21 = (1u << 21) - 1;
  const int32_t off = 1 << 20;
  for (size_t g = 0; g < o.claims.size(); ++g)
    for (auto& kv : o.claims[g]) {
      grain[k] = (int32_t)g;
      site[3 * k + 0] = (int32_t)((kv.first >> 42) & m21) - off;
      site[3 * k + 1] = (int32_t)((kv.first >> 21) & m21) - off;
      site[3 * k + 2] = (int32_t)(kv.first & m21) - off;
      flags[k] = kv.second;
      ++k;
    }
}

void orc_get_sites(void* h, int32_t* state) {
  Oracle& o = *(Oracle*)h;
  for (size_t i = 0; i < o.sites.size(); ++i) state[i] = o.sites[i].state;
}

// Replaces the dynamic state: grains (centre, quaternion), particles
// (grain, site, dir, s, state; positions rebuilt on the lattice), claims,
// site states, time and step.
int32_t orc_load_state(void* h, int32_t n_grains, const double* centre, const double* quat,
                       int64_t n_parts, const int32_t* grain, const int32_t* site,
                       const int32_t* dir, const double* s, const int32_t* state,
                       int64_t n_claims, const int32_t* c_grain, const int32_t* c_site,
                       const uint8_t* c_flags, int32_t n_sites, const int32_t* site_state,
                       double t, int64_t step) {
  Oracle& o = *(Oracle*)h;
  o.grains.clear();
  o.claims.clear();
  o.parts.clear();
  o.grain_site.clear();
  // A grain whose centre is a fired site's position came from that site.
  for (int32_t g = 0; g < n_grains; ++g) {
    int32_t from = -1;
    for (size_t i = 0; i < o.sites.size() && i < (size_t)n_sites && from < 0; ++i)
      if (site_state[i] == S_FIRED && o.sites[i].y[0] == centre[3 * g] &&
          o.sites[i].y[1] == centre[3 * g + 1] && o.sites[i].y[2] == centre[3 * g + 2])
        from = (int32_t)i;
    add_grain(o, centre + 3 * g, quat + 4 * g, from);
  }
  o.parts.resize(n_parts);
  for (int64_t i = 0; i < n_parts; ++i) {
    Particle& q = o.parts[i];
    q.g = grain[i];
    if (q.g < 0 || q.g >= n_grains) return E_INVAL;
    for (int a = 0; a < 3; ++a) q.site[a] = site[3 * i + a];
    q.dir = dir[i];
    q.s = s[i];
    q.state = state[i];
    lattice_position(o.p, o.grains[q.g], q.site, q.dir, q.s, q.x);
  }
  for (int64_t k = 0; k < n_claims; ++k) {
    if (c_grain[k] < 0 || c_grain[k] >= n_grains) return E_INVAL;
    add_claim(o.claims[c_grain[k]], c_site + 3 * k, c_flags[k]);
  }
  if (n_sites != (int32_t)o.sites.size()) return E_INVAL;
  for (int32_t i = 0; i < n_sites; ++i) o.sites[i].state = site_state[i];
  o.t = t;
  o.step = step;
  o.err = E_OK;
  return E_OK;
}

// Grain map (Sec. 2.3): voxel centre y = origin + (i + 1/2) spacing gets
// label g + 1 when the rounded lattice position of y in grain g is a reached
// site; among several such grains the smallest distance to that site wins,
// then the lower grain index.  0 = liquid.
void orc_grain_map(void* h, const int32_t n[3], const double origin[3], const double spacing[3],
                   uint32_t* out) {
  Oracle& o = *(Oracle*)h;
  const int64_t total = (int64_t)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t v = 0; v < total; ++v) {
    int64_t i = v % n[0], j = (v / n[0]) % n[1], k = v / ((int64_t)n[0] * n[1]);
    double y[3] = {origin[0] + (i + 0.5) * spacing[0], origin[1] + (j + 0.5) * spacing[1],
                   origin[2] + (k + 0.5) * spacing[2]};
    uint32_t best = 0;
    double bd = INFINITY;
    for (size_t g = 0; g < o.grains.size(); ++g)
      for (int k = 0; k < 27; ++k) {
        // The voxel centre and, on periodic axes, its images.
        const int sh[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
        bool ok = true;
        double yi[3];
        for (int a = 0; a < 3; ++a) {
          if (sh[a] != 0 && !periodic_axis(o.p, a)) ok = false;
          yi[a] = y[a] + sh[a] * (o.p.hi[a] - o.p.lo[a]);
        }
        if (!ok) continue;
        int32_t s[3];
        lattice_round(o.p, o.grains[g], yi, s);
        auto it = o.claims[g].find(site_key(s[0], s[1], s[2]));
        if (it == o.claims[g].end() || !(it->second & C_REACHED)) continue;
        double ps[3];
        lattice_position(o.p, o.grains[g], s, 0, 0.0, ps);
        double d = dist2(yi, ps);
        if (d < bd) { bd = d; best = (uint32_t)g + 1; }
      }
    out[v] = best;
  }
}

// ------------------------------------------------- FP32 checker ----------
// Single-rounded FP32 binning: cell = (int)floorf((x - lo) * inv_h), one FP32
// subtract and one FP32 multiply, clamped to [0, n-1].
// Mushy-zone deposition (reading R14).  The inside of a grain's envelope is
// the set of lattice sites the grain has reached, each standing for its
// crystal-frame cube of edge lambda0 (the mushy zone of Sec. 2.2 is the
// volume inside the envelopes).  A reached site counts in the node-centred
// cell of the grid (n, origin, spacing) that holds its centre,
// index floor((x - origin) / spacing + 1/2) per axis; sites outside every
// cell are not counted.  FP64.
void orc_deposit_counts(void* h, const int32_t n[3], const double origin[3],
                        const double spacing[3], uint32_t* out) {
  Oracle& o = *(Oracle*)h;
  std::fill(out, out + (size_t)n[0] * n[1] * n[2], 0u);
  const uint64_t m21 = (1u << 21) - 1;
  const int32_t off = 1 << 20;
  for (size_t g = 0; g < o.claims.size(); ++g) {
    const Grain& G = o.grains[g];
    for (auto& kv : o.claims[g]) {
      if (!(kv.second & C_REACHED)) continue;
      const double S[3] = {(double)((int32_t)((kv.first >> 42) & m21) - off),
                           (double)((int32_t)((kv.first >> 21) & m21) - off),
                           (double)((int32_t)(kv.first & m21) - off)};
      int64_t idx[3];
      bool in = true;
      double x[3], xw[3];
      for (int a = 0; a < 3; ++a)
        x[a] = G.c[a] + o.p.lambda0 * (G.R[a][0] * S[0] + G.R[a][1] * S[1] + G.R[a][2] * S[2]);
      wrap_pos(o.p, x, xw);
      for (int a = 0; a < 3; ++a) {
        const double f = std::floor((xw[a] - origin[a]) / spacing[a] + 0.5);
        if (!(f >= 0 && f < n[a])) in = false;
        idx[a] = (int64_t)f;
      }
      if (in) ++out[((size_t)idx[2] * n[1] + idx[1]) * n[0] + idx[0]];
    }
  }
}

// FP32 checker of the deposition: the site centre computed from FP32 grain
// rows (centre at [0..2], lambda0 R row-major at [13..21]) as a chain of
// single-rounded fused multiply-adds, x = c + (lR)_{a0} S0 + (lR)_{a1} S1 +
// (lR)_{a2} S2 taken from the S2 term outwards, and the index
// floor((x - origin) * inv_spacing + 1/2) with each operation rounded to FP32.
void orc_f32_deposit(int64_t m, const int32_t* grain, const int32_t* site, const float* gtab,
                     const int32_t n[3], const float origin[3], const float inv_sp[3],
                     uint32_t* out) {
  std::fill(out, out + (size_t)n[0] * n[1] * n[2], 0u);
  for (int64_t k = 0; k < m; ++k) {
    const float* G = gtab + (size_t)grain[k] * 24;
    const float f0 = (float)site[3 * k], f1 = (float)site[3 * k + 1], f2 = (float)site[3 * k + 2];
    int64_t idx[3];
    bool in = true;
    for (int a = 0; a < 3; ++a) {
      const float* row = G + 13 + 3 * a;
      const float x = fmaf(row[0], f0, fmaf(row[1], f1, fmaf(row[2], f2, G[a])));
      volatile float d = x - origin[a];
      volatile float u = d * inv_sp[a];
      volatile float v = u + 0.5f;
      const float f = floorf(v);
      if (!(f >= 0.0f && f < (float)n[a])) in = false;
      idx[a] = (int64_t)f;
    }
    if (in) ++out[((size_t)idx[2] * n[1] + idx[1]) * n[0] + idx[0]];
  }
}

void orc_f32_cells(int64_t n, const float* xyz, const float lo[3], float inv_h,
                   const int32_t ncell[3], int32_t* out) {
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      volatile float d = xyz[3 * i + a] - lo[a];
      volatile float u = d * inv_h;
      float fl = floorf(u);
      int32_t c;
      if (fl < 0.0f) c = 0;
      else if (fl > (float)(ncell[a] - 1)) c = ncell[a] - 1;
      else c = (int32_t)fl;
      out[3 * i + a] = c;
    }
}

// FP32 containment decisions on given FP32 positions: particle i with role 1
// (active) stops when some particle j with role 1 or 2 (stopped) of another
// grain has d2 < rc2, d2 = (dx*dx + dy*dy) + dz*dz in single-rounded FP32.
// Candidate pairs come from a grid of cells of edge 2*sqrt(rc2), so no pair
// within rc is missed whatever the rounding.
void orc_f32_contain(int64_t n, const float* xyz, const int32_t* grain, const uint8_t* role,
                     float rc2, uint8_t* out) {
  double cs = 2.0 * std::sqrt((double)rc2);
  std::unordered_map<int64_t, std::vector<int64_t>> cells;
  auto key = [](int64_t i, int64_t j, int64_t k) {
    return ((i + (1 << 20)) << 42) ^ ((j + (1 << 20)) << 21) ^ (k + (1 << 20));
  };
  std::vector<int64_t> ci(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) ci[3 * i + a] = (int64_t)std::floor((double)xyz[3 * i + a] / cs);
    if (role[i]) cells[key(ci[3 * i], ci[3 * i + 1], ci[3 * i + 2])].push_back(i);
  }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    out[i] = 0;
    if (role[i] != 1) continue;
    bool hit = false;
    for (int dk = -1; dk <= 1 && !hit; ++dk)
      for (int dj = -1; dj <= 1 && !hit; ++dj)
        for (int di = -1; di <= 1 && !hit; ++di) {
          auto it = cells.find(key(ci[3 * i] + di, ci[3 * i + 1] + dj, ci[3 * i + 2] + dk));
          if (it == cells.end()) continue;
          for (int64_t j : it->second) {
            if (grain[j] == grain[i]) continue;
            volatile float dx = xyz[3 * i] - xyz[3 * j];
            volatile float dy = xyz[3 * i + 1] - xyz[3 * j + 1];
            volatile float dz = xyz[3 * i + 2] - xyz[3 * j + 2];
            volatile float xx = dx * dx;
            volatile float yy = dy * dy;
            volatile float zz = dz * dz;
            volatile float sxy = xx + yy;
            volatile float d2 = sxy + zz;
            if (d2 < rc2) { hit = true; break; }
          }
        }
    out[i] = hit ? 1 : 0;
  }
}

// --------------------------------------------------- adjoint (FP64) ------
// Frozen-mask forward: runs n_steps ordinary steps (branching must be off and
// no sites registered) and records for each particle present at the start the
// number of steps in which it advanced.
int32_t orc_adjoint_record(void* h, double dt, int32_t n_steps, int32_t* nact) {
  Oracle& o = *(Oracle*)h;
  if (o.p.branching) return E_INVAL;
  for (auto& s : o.sites) if (s.state == S_DORMANT) return E_INVAL;
  const size_t n0 = o.parts.size();
  for (size_t i = 0; i < n0; ++i) nact[i] = 0;
  for (int32_t k = 0; k < n_steps; ++k) {
    for (size_t i = 0; i < n0; ++i) nact[i] += o.parts[i].state == P_ACTIVE ? 1 : 0;
    do_step(o, dt);
    if (o.err != E_OK) return o.err;
  }
  return E_OK;
}

// Replay of one particle with frozen mask: s advances in steps k < nact only.
// Returns s after n_steps; if `trace` is non-null it receives s_k, k = 0..n_steps.
static double replay_one(const Oracle& o, const Params& p, const Grain& g, const int32_t site[3],
                         int d, double s0, int32_t nact, double t0, double dt, int32_t n_steps,
                         double* trace) {
  double s = s0;
  if (trace) trace[0] = s;
  for (int32_t k = 0; k < n_steps; ++k) {
    if (k < nact) {
      double x[3], xw[3];
      lattice_position(p, g, site, d, s, x);
      wrap_pos(p, x, xw);
      double dT = field_value(o.f, xw, t0 + k * dt) - p.theta;
      s += velocity(p, dT) * dt;
    }
    if (trace) trace[k + 1] = s;
  }
  return s;
}

// Positions after n_steps of frozen-mask replay with kinetics a[2] and offset
// theta; particles are given explicitly (grain, site, dir, s0, nact).
int32_t orc_adjoint_replay(void* h, const double a[2], double theta, int64_t n,
                           const int32_t* grain, const int32_t* site, const int32_t* dir,
                           const double* s0, const int32_t* nact, double t0, double dt,
                           int32_t n_steps, double* xN) {
  Oracle& o = *(Oracle*)h;
  Params p = o.p;
  p.a[0] = a[0]; p.a[1] = a[1]; p.theta = theta;
  if (o.f.kind == F_ROSENTHAL) return E_INVAL;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const Grain& g = o.grains[grain[i]];
    double s = replay_one(o, p, g, site + 3 * i, dir[i], s0[i], nact[i], t0, dt, n_steps, nullptr);
    lattice_position(p, g, site + 3 * i, dir[i], s, xN + 3 * i);
  }
  return E_OK;
}

// Reverse-mode gradient of  sum_i <dLdx_i, x_i^N>  with respect to
// (a[0], a[1], theta) under frozen masks.  Per particle, with u = R e_d and
// x = x_site + s u:  lambda_N = <dLdx, u>;  for k = N-1 .. 0 with the particle
// active:  grad_a_j += lambda_{k+1} dt dT_k^b_j (dT_k > 0),
// grad_theta -= lambda_{k+1} dt v'(dT_k),
// lambda_k = lambda_{k+1} (1 + dt v'(dT_k) <grad F(x_k), u>).
int32_t orc_adjoint_grad(void* h, int64_t n, const int32_t* grain, const int32_t* site,
                         const int32_t* dir, const double* s0, const int32_t* nact, double t0,
                         double dt, int32_t n_steps, const double* dLdx, double grad[3]) {
  Oracle& o = *(Oracle*)h;
  const Params& p = o.p;
  if (o.f.kind == F_ROSENTHAL) return E_INVAL;
  double G0 = 0, G1 = 0, G2 = 0;
#pragma omp parallel for schedule(static) reduction(+ : G0, G1, G2)
  for (int64_t i = 0; i < n; ++i) {
    const Grain& g = o.grains[grain[i]];
    std::vector<double> tr((size_t)n_steps + 1);
    replay_one(o, p, g, site + 3 * i, dir[i], s0[i], nact[i], t0, dt, n_steps, tr.data());
    double u[3];
    direction(g, dir[i], u);
    double lam = dLdx[3 * i] * u[0] + dLdx[3 * i + 1] * u[1] + dLdx[3 * i + 2] * u[2];
    for (int32_t k = n_steps - 1; k >= 0; --k) {
      if (k >= nact[i]) continue;
      double x[3], xw[3], gF[3];
      lattice_position(p, g, site + 3 * i, dir[i], tr[k], x);
      wrap_pos(p, x, xw);
      double dT = field_value(o.f, xw, t0 + k * dt, gF) - p.theta;
      double vp = velocity_slope(p, dT);
      if (dT > 0) {
        G0 += lam * dt * std::pow(dT, p.b[0]);
        G1 += lam * dt * std::pow(dT, p.b[1]);
      }
      G2 -= lam * dt * vp;
      double du = gF[0] * u[0] + gF[1] * u[1] + gF[2] * u[2];
      lam = lam * (1 + dt * vp * du);
    }
  }
  grad[0] = G0;
  grad[1] = G1;
  grad[2] = G2;
  return E_OK;
}

}  // extern "C"
