// TPC track-reconstruction ORACLE -- test infrastructure only.
//
// A plain, slow, single-threaded CPU implementation of the tracking method:
// cellular-automaton seeding (neighbour links on adjacent pad rows, mutual
// cleaning, chains of >= 3 clusters) followed by Kalman-filter track following,
// max-key hit arbitration, track selection, a Kalman refit and the merge of
// track pieces across neighbouring sectors.  The paper (section 5: full TPC
// tracking of every collision is required for track-model compression;
// section 6: TPC tracking is the critical GPU step) states THAT this is
// computed but not HOW; every algorithmic constant and step below is a reading
// of the method written out explicitly, and the numbered "O" steps refer to
// that reading (O1 frame/track model, O2 helix propagation, O3 grid (not
// needed here: rows are searched in full or by binary search in z), O4
// neighbours, O5 cleaning, O6 starts, O7 tracklets, O8 Kalman update,
// O9 selection and fit, A13 downward extension, O10 merge, A21 central-membrane merge,
// A25 pairing of a looper's two legs), C1-C5 for the track-model compression that
// consumes the tracks, E1-E5 for the rANS entropy coder after it, and F1-F6 for the
// cluster finding before the tracking (section 5).
//
// Only tests/, the smoke check and the CPU baseline leg of the benchmark may
// load this library.  It shares no code, header, table or constant generator
// with the HIP library.
//
// Two builds of every numerical step exist through one template:
//   * float  -- the "FP32 mirror": the exact operation order that defines the
//               bit-exact outputs (links, tracklet hits, track hit lists).
//               Compile with -ffp-contract=off and without -ffast-math.
//   * double -- the FP64 refit used as the reference for fitted parameters;
//               its asin comes from libm.
//
// Pins (tests/): helix propagation against the closed-form circle and an RK4
// integration of the Lorentz force; the propagation Jacobian against central
// finite differences; the Kalman update against the information-form identity;
// the FP32 asin(u)/u series against libm; neighbour links against a
// brute-force triple search; chain/ownership invariants; zero-smear fits
// recovering the truth; the downward extension (A13) recovering every lower cluster of
// tracks whose chains cannot start below a row, its miss limit, and the rule for
// clusters found by two tracks; the two legs of exact loopers paired with each other and with
// nothing across events or with one curvature flipped, and on a full event every pair joining
// both legs of one particle; the window searches over the z range of a row against scans of
// the whole row.  The hit-picking heuristic of the tracklet following
// (O7 window search), of the extension's window search (A13) and the merge pairing
// (O10) are pinned only by invariants and special cases: parity unpinned beyond those.  Compression: the prediction
// against an FP64 closed-form circle in the rotated frame, zero residual codes for
// clusters placed exactly on the fitted helix, absolute codes against numpy's rint,
// and the round trip within half a quantisation step.  Cluster finding: exact centroids
// of symmetric and hand-computed charge patterns, the tie rule, translation invariance,
// and the generator's clusters recovered from its digits.  rANS: exact round trips, the
// model's normalisation rule and closed forms, lane sizes within a few words of the
// information content under the model.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace {

constexpr int kRows = 152;
constexpr int kSectors = 36;
constexpr int kRowsPerSide = 18;

// ---------------------------------------------------------------- parameters
// Layout mirrored by oracle/oracle.py (ctypes).  Every float is used as is in
// FP32; derived FP32 constants are formed in double and rounded once.
struct Params {
  float win_dy_slope, win_dy_const, win_dz_slope, win_dz_const;  // O4 up window
  float link_cut;                                                // O4 second-difference cut
  float cy0, cz0, cs0, ct0, ck0;                                 // O7 tracklet priors
  float cy1, cz1, cs1, ct1, ck1;                                 // O9 fit priors
  float sigma_y, sigma_z;                                        // O8 measurement errors
  float nwin, chi2_follow;                                       // O7 following
  int32_t max_miss, min_hits;
  float smax;                                                    // |sin phi| limit
  float bz;                                                      // field, tesla
  float merge_edge, chi2_merge;                                  // O10
  float merge_dz;                                                // O10 z gate
  float v_drift;                                                 // T1 drift velocity, cm/us
  int32_t ext_down;                                              // A13 downward extension (0: off)
  int32_t merge_membrane;                                        // A21 central-membrane merge (0: off)
};

// Pad-row plane positions (O1, reading A2): x_r = 85 + r * 160/151 cm, rounded once.
struct Geometry {
  float x[kRows];
  float cos20, sin20, tan10;
  Geometry() {
    for (int r = 0; r < kRows; ++r) x[r] = (float)(85.0 + (double)r * 160.0 / 151.0);
    const double a = 20.0 * 3.14159265358979323846 / 180.0;
    cos20 = (float)std::cos(a);
    sin20 = (float)std::sin(a);
    tan10 = (float)std::tan(a / 2.0);
  }
};
const Geometry kGeo;

// Signed curvature per unit q/pT: C = -kappa * B * (q/pT), kappa = 0.299792458e-2 GeV/(T cm).
template <class T> T curvature_factor(const Params& p) {
  return (T)(-0.299792458e-2 * (double)p.bz);
}

// ---------------------------------------------------------------- asin(u)/u
// A(u) = asin(u)/u and B(u) = A'(u)/u.  FP32: Taylor coefficients of asin,
// Horner in w = u^2 for |u| <= 1/2 (relative truncation error < 2^-25); above,
// asin(u) = pi/2 - 2 asin(sqrt((1-|u|)/2)).  FP64: libm.
const float kA[10] = {0x1p+0f,         0x1.555556p-3f, 0x1.333334p-4f, 0x1.6db6dcp-5f,
                      0x1.f1c71cp-6f,  0x1.6e8ba2p-6f, 0x1.1c4ec4p-6f, 0x1.c9999ap-7f,
                      0x1.7a8788p-7f,  0x1.3fde50p-7f};
const float kB[12] = {0x1.555556p-2f, 0x1.333334p-2f, 0x1.124924p-2f, 0x1.f1c71cp-3f,
                      0x1.ca2e8cp-3f, 0x1.aa7628p-3f, 0x1.906666p-3f, 0x1.7a8788p-3f,
                      0x1.67da1ap-3f, 0x1.57ab0cp-3f, 0x1.497922p-3f, 0x1.3ce4aep-3f};

float series_A(float w) {
  float a = kA[9];
  for (int i = 8; i >= 0; --i) a = kA[i] + w * a;
  return a;
}
float series_B(float w) {
  float b = kB[11];
  for (int i = 10; i >= 0; --i) b = kB[i] + w * b;
  return b;
}

void asinc(float u, float& A, float& B) {
  const float au = std::fabs(u);
  const float w = u * u;
  if (au <= 0.5f) {
    A = series_A(w);
    B = series_B(w);
  } else {
    const float v = std::sqrt((1.0f - au) * 0.5f);
    const float asn = 0x1.921fb6p+0f - 2.0f * (v * series_A(v * v));
    A = asn / au;
    const float g = 1.0f / std::sqrt((1.0f - u) * (1.0f + u));
    B = (g - A) / w;
  }
}

void asinc(double u, double& A, double& B) {
  const double au = std::fabs(u);
  const double w = u * u;
  if (au < 0.05) {
    // a_n = C(2n,n) / (4^n (2n+1)); B(u) = sum 2(n+1) a_{n+1} w^n
    double an[9];
    for (int n = 0; n < 9; ++n) {
      double c = 1.0;
      for (int i = 1; i <= n; ++i) c = c * (double)(n + i) / (double)(4 * i);
      an[n] = c / (double)(2 * n + 1);
    }
    A = 0.0;
    for (int n = 7; n >= 0; --n) A = an[n] + w * A;
    B = 0.0;
    for (int n = 7; n >= 0; --n) B = 2.0 * (double)(n + 1) * an[n + 1] + w * B;
  } else {
    A = std::asin(au) / au;
    B = (1.0 / std::sqrt((1.0 - u) * (1.0 + u)) - A) / w;
  }
}

// ---------------------------------------------------------------- track state
// O1: state at a pad-row plane x: P = (y, z, s = sin phi, t = tan lambda, k = q/pT);
// covariance stored as the lower triangle, index(i,j) = i(i+1)/2 + j, j <= i.
inline int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

template <class T> bool all_finite(const T* P, const T* C) {
  for (int i = 0; i < 5; ++i)
    if (!(P[i] - P[i] == T(0))) return false;
  for (int i = 0; i < 15; ++i)
    if (!(C[i] - C[i] == T(0))) return false;
  return true;
}

// The state vector is carried as an unevaluated sum hi + lo per component
// (compensated accumulation): every increment is added with an exact two-sum and
// the rounding error is kept in lo.  This keeps FP32 increments of 1e-3..1e-6
// from being lost against O(1..100) state values.  hi is always fl(hi + lo).
template <class T> inline void acc(T& hi, T& lo, T d) {
  const T s = hi + d;
  const T bb = s - hi;
  const T e = (hi - (s - bb)) + (d - bb);
  const T t = lo + e;
  hi = s + t;
  lo = t - (hi - s);
}

// O2: exact helix transport from plane x1 to plane x2 on the branch cos(phi) > 0,
// with the analytic Jacobian J and C' = J C J^T.  Returns false on failure
// (|s2| >= smax or |u| >= 1), leaving P and C untouched.
template <class T>
bool propagate(T* P, T* L, T* C, T x1, T x2, T cb, T smax) {
  const T dx = x2 - x1;
  if (dx == T(0)) return true;
  const T curv = P[4] * cb;
  const T s1 = P[2];
  const T s2 = s1 + curv * dx;
  if (!(std::fabs(s2) < smax)) return false;
  const T c1 = std::sqrt((T(1) - s1) * (T(1) + s1));
  const T c2 = std::sqrt((T(1) - s2) * (T(1) + s2));
  const T cc = c1 + c2;
  const T f = (s1 + s2) / cc;
  const T dy = dx * f;
  T ch = std::sqrt(dx * dx + dy * dy);
  if (dx < T(0)) ch = -ch;
  const T u = curv * ch * T(0.5);
  if (!(std::fabs(u) < T(1))) return false;
  T A, B;
  asinc(u, A, B);
  const T g = T(1) / std::sqrt((T(1) - u) * (T(1) + u));
  const T dS = ch * A;
  // Jacobian entries (all others are those of the identity)
  const T q1 = s1 / c1;
  const T q2 = s2 / c2;
  const T fs = (T(2) + f * (q1 + q2)) / cc;
  const T fc = dx * (T(1) + f * q2) / cc;
  const T ja = dx * fs;                                  // dy / ds1
  const T jb = dx * fc * cb;                             // dy / dk
  const T chs = dy * ja / ch;
  const T chk = dy * jb / ch;
  const T dSs = g * chs;
  const T dSk = g * chk + ch * ch * u * B * T(0.5) * cb;
  const T t = P[3];
  const T je = t * dSs;                                  // dz / ds1
  const T jf = dS;                                       // dz / dt
  const T jg = t * dSk;                                  // dz / dk
  const T jh = cb * dx;                                  // ds2 / dk
  // state
  acc(P[0], L[0], dy);
  acc(P[1], L[1], t * dS);
  acc(P[2], L[2], curv * dx);
  // covariance: M = J C, then C' = M J^T (lower triangle)
  T c[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) c[i][j] = C[tri(i, j)];
  T M[5][5];
  for (int j = 0; j < 5; ++j) {
    M[0][j] = c[0][j] + ja * c[2][j] + jb * c[4][j];
    M[1][j] = c[1][j] + je * c[2][j] + jf * c[3][j] + jg * c[4][j];
    M[2][j] = c[2][j] + jh * c[4][j];
    M[3][j] = c[3][j];
    M[4][j] = c[4][j];
  }
  for (int i = 0; i < 5; ++i) {
    const T n0 = M[i][0] + ja * M[i][2] + jb * M[i][4];
    const T n1 = M[i][1] + je * M[i][2] + jf * M[i][3] + jg * M[i][4];
    const T n2 = M[i][2] + jh * M[i][4];
    const T n3 = M[i][3];
    const T n4 = M[i][4];
    const T n[5] = {n0, n1, n2, n3, n4};
    for (int j = 0; j <= i; ++j) C[tri(i, j)] = n[j];
  }
  return true;
}

// O8: the inverse of the 2x2 innovation covariance S = C[0:2,0:2] + diag(vy, vz).
template <class T> struct SInv {
  T i00, i10, i11;
  bool ok;
};
template <class T> SInv<T> s_inverse(const T* C, T vy, T vz) {
  SInv<T> r;
  const T S00 = C[0] + vy;
  const T S10 = C[1];
  const T S11 = C[2] + vz;
  const T det = S00 * S11 - S10 * S10;
  r.ok = det > T(0);
  const T idet = T(1) / det;
  r.i00 = S11 * idet;
  r.i10 = -(S10 * idet);
  r.i11 = S00 * idet;
  return r;
}
template <class T> T chi2_of(const SInv<T>& s, T r0, T r1) {
  const T a0 = s.i00 * r0 + s.i10 * r1;
  const T a1 = s.i10 * r0 + s.i11 * r1;
  return r0 * a0 + r1 * a1;
}

// O8: Kalman update with the measurement (my, mz).  Returns false (state untouched)
// if det <= 0, any value becomes non-finite, or |s| >= smax.
template <class T>
bool kf_update(T* P, T* L, T* C, T my, T mz, T vy, T vz, T smax, T* chi2_out) {
  const SInv<T> si = s_inverse(C, vy, vz);
  if (!si.ok) return false;
  const T r0 = (my - P[0]) - L[0];
  const T r1 = (mz - P[1]) - L[1];
  const T chi2 = chi2_of(si, r0, r1);
  T c0[5], c1[5];
  for (int i = 0; i < 5; ++i) {
    c0[i] = C[tri(i, 0)];
    c1[i] = C[tri(i, 1)];
  }
  T K0[5], K1[5];
  for (int i = 0; i < 5; ++i) {
    K0[i] = c0[i] * si.i00 + c1[i] * si.i10;
    K1[i] = c0[i] * si.i10 + c1[i] * si.i11;
  }
  T Pn[5], Ln[5], Cn[15];
  for (int i = 0; i < 5; ++i) {
    Pn[i] = P[i];
    Ln[i] = L[i];
    acc(Pn[i], Ln[i], K0[i] * r0 + K1[i] * r1);
  }
  // Rows/columns of the measured components use the exact identity
  // C'(i,m) = C(i,:m) S^-1 V = K(i,m) V (no cancellation); the rest is C - K H C.
  for (int i = 0; i < 5; ++i) {
    Cn[tri(i, 0)] = K0[i] * vy;
    if (i >= 1) Cn[tri(i, 1)] = K1[i] * vz;
    for (int j = 2; j <= i; ++j)
      Cn[tri(i, j)] = C[tri(i, j)] - (K0[i] * c0[j] + K1[i] * c1[j]);
  }
  if (!all_finite(Pn, Cn)) return false;
  if (!(std::fabs(Pn[2]) < smax)) return false;
  std::memcpy(P, Pn, sizeof(Pn));
  std::memcpy(L, Ln, sizeof(Ln));
  std::memcpy(C, Cn, sizeof(Cn));
  if (chi2_out) *chi2_out = chi2;
  return true;
}

// ---------------------------------------------------------------- the oracle
struct Tracklet {
  int32_t start;              // original index of the first chain cluster
  int32_t n;                  // hits
  bool valid;                 // n >= min_hits
  std::vector<int32_t> hits;  // original indices, rows ascending
  float P[5], C[15], x;       // state at the last hit (after its update)
};

struct Track {
  int32_t tracklet;           // tracklet id it was selected from (== track id)
  int32_t job, sector, event;
  std::vector<int32_t> hits;  // original indices, inner -> outer
  float P[5], C[15], x, chi2; int32_t ndf;   // FP32 fit at the innermost hit
  float L[5];                 // its compensation terms (the low parts of P)
  int32_t n_ext = 0;          // hits gained by the downward extension (A13)
  float link_t0 = NAN;        // A21: collision time of the membrane link to the outer partner
  float t0m = NAN;            // A21: a chain head's collision time from its membrane link
  double Pd[5], Cd[15], xd, chi2d; int32_t ndfd;   // FP64 refit
  // merge bookkeeping: a merged track keeps the inner piece's id; the outer piece is absorbed
  int32_t merged_into = -1;
  int32_t partner = -1;
  int32_t sector2 = -1;       // sector of the last absorbed outer piece, -1 if none
  std::vector<int32_t> pieces;  // chain head: its absorbed pieces, inner -> outer
};

// O10: re-express a state in the frame of the adjacent sector `to` (same side; the
// sector angle changes by d = +-20 degrees).  The point keeps its global position:
// x' = x cos d + y sin d, y' = -x sin d + y cos d; the direction turns by -d:
// s' = s cos d - c sin d, c' = c cos d + s sin d; z, t, k are unchanged.  The new
// reference plane is x' = const, so a shift dy of y at fixed x moves the point by
// dy sin d off that plane; moving it back along the helix by dx' = -dy sin d changes
// y' by dx' s'/c', z by dx' t/c' and sin(phi) by dx' times the curvature k cb:
// dy'/dy = (cos d c' - sin d s')/c' = c/c', dz'/dy = -t sin d / c',
// ds'/dy = -k cb sin d.  A change of s at fixed point turns only the direction:
// ds'/ds = cos d + sin d s/c = c'/c.  Fails unless c' > 0 and |s'| < smax.
template <class T> bool rotate_sector(T* P, T* L, T* C, T& x, int from, int to, T cb, T smax) {
  const int df = ((to % kRowsPerSide) - (from % kRowsPerSide) + kRowsPerSide) % kRowsPerSide;
  if (df != 1 && df != kRowsPerSide - 1) return false;
  const T ca = (T)kGeo.cos20;
  const T sa = df == 1 ? (T)kGeo.sin20 : -(T)kGeo.sin20;
  const T s = P[2];
  const T c = std::sqrt((T(1) - s) * (T(1) + s));
  const T xn = x * ca + P[0] * sa;
  const T yn = P[0] * ca - x * sa;
  const T sn = s * ca - c * sa;
  const T cn = c * ca + s * sa;
  if (!(cn > T(0)) || !(std::fabs(sn) < smax)) return false;
  const T ja = c / cn;                 // dy'/dy
  const T jb = -(P[3] * sa / cn);      // dz'/dy
  const T jc = -(P[4] * cb * sa);      // ds'/dy
  const T je = cn / c;                 // ds'/ds
  T c5[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) c5[i][j] = C[tri(i, j)];
  T M[5][5];
  for (int j = 0; j < 5; ++j) {
    M[0][j] = ja * c5[0][j];
    M[1][j] = jb * c5[0][j] + c5[1][j];
    M[2][j] = jc * c5[0][j] + je * c5[2][j];
    M[3][j] = c5[3][j];
    M[4][j] = c5[4][j];
  }
  for (int i = 0; i < 5; ++i) {
    const T n[5] = {ja * M[i][0], jb * M[i][0] + M[i][1], jc * M[i][0] + je * M[i][2], M[i][3], M[i][4]};
    for (int j = 0; j <= i; ++j) C[tri(i, j)] = n[j];
  }
  P[0] = yn;
  P[2] = sn;
  L[0] = T(0);
  L[2] = T(0);
  x = xn;
  return all_finite(P, C);
}

struct Oracle {
  Params p;
  int32_t n = 0, J = 0;
  std::vector<uint8_t> sector;
  std::vector<int16_t> row;
  std::vector<float> y, z;
  std::vector<int32_t> job_off, job_of, job_event;
  std::vector<uint8_t> valid;
  int32_t status = 0;  // bit 0: a cluster with an out-of-range field was excluded

  // row lists: clusters of (job, sector, row), sorted by (z, index)
  std::vector<int64_t> slot_off;
  std::vector<int32_t> slot_idx;

  std::vector<int32_t> up_raw, down_raw, up, down;
  std::vector<int32_t> starts;
  std::vector<Tracklet> tracklets;
  std::vector<uint64_t> hitw;
  std::vector<Track> tracks;      // selected, in tracklet-id order
  bool brute = false;             // search whole rows instead of the z-sorted range
  double fp64_seconds = 0.0;      // wall time spent in the FP64 refits (timing only)

  int64_t slot(int j, int s, int r) const { return ((int64_t)j * kSectors + s) * kRows + r; }

  // -------- O3: group clusters by (job, sector, row) -- the search structure
  void build_rows() {
    const int64_t ns = (int64_t)J * kSectors * kRows;
    slot_off.assign(ns + 1, 0);
    std::vector<int64_t> key(n, -1);
    for (int32_t i = 0; i < n; ++i) {
      if (!valid[i]) continue;
      key[i] = slot(job_of[i], sector[i], row[i]);
      slot_off[key[i] + 1]++;
    }
    for (int64_t s = 0; s < ns; ++s) slot_off[s + 1] += slot_off[s];
    slot_idx.assign(slot_off[ns], 0);
    std::vector<int64_t> fill(slot_off.begin(), slot_off.end() - 1);
    for (int32_t i = 0; i < n; ++i)
      if (key[i] >= 0) slot_idx[fill[key[i]]++] = i;
    for (int64_t s = 0; s < ns; ++s)
      std::sort(slot_idx.begin() + slot_off[s], slot_idx.begin() + slot_off[s + 1],
                [&](int32_t a, int32_t b) { return z[a] < z[b] || (z[a] == z[b] && a < b); });
  }

  // index range [lo, hi) of slot s whose z lies in [zlo, zhi]
  void z_range(int64_t s, float zlo, float zhi, int64_t& lo, int64_t& hi) const {
    lo = slot_off[s];
    hi = slot_off[s + 1];
    if (brute) return;
    const int32_t* b = slot_idx.data();
    lo = std::lower_bound(b + lo, b + hi, zlo, [&](int32_t i, float v) { return z[i] < v; }) - b;
    hi = std::upper_bound(b + lo, b + hi, zhi, [&](float v, int32_t i) { return v < z[i]; }) - b;
  }

  // -------- O4: neighbour links
  void find_neighbours() {
    up_raw.assign(n, -1);
    down_raw.assign(n, -1);
    const float cut2 = p.link_cut * p.link_cut;
    const float zmargin = 0.01f;
    for (int32_t h = 0; h < n; ++h) {
      if (!valid[h]) continue;
      const int r = row[h], s = sector[h], j = job_of[h];
      const float yh = y[h], zh = z[h];
      for (int d = 1; d <= 2; ++d) {
        if (r - d < 0 || r + d >= kRows) break;
        const float dxu = kGeo.x[r + d] - kGeo.x[r];
        const float wy = p.win_dy_slope * dxu + p.win_dy_const;
        const float wz = p.win_dz_slope * dxu + p.win_dz_const;
        const float rho = kGeo.x[r + d] / kGeo.x[r];
        const float yc = yh * rho;
        float best = 0.f;
        int32_t bu = -1, bd = -1;
        int64_t ulo, uhi;
        z_range(slot(j, s, r + d), zh - wz - zmargin, zh + wz + zmargin, ulo, uhi);
        for (int64_t a = ulo; a < uhi; ++a) {
          const int32_t u = slot_idx[a];
          if (!(std::fabs(y[u] - yc) <= wy) || !(std::fabs(z[u] - zh) <= wz)) continue;
          const float pz = (zh + zh) - z[u];
          int64_t dlo, dhi;
          z_range(slot(j, s, r - d), pz - p.link_cut - zmargin, pz + p.link_cut + zmargin, dlo, dhi);
          for (int64_t b = dlo; b < dhi; ++b) {
            const int32_t dd = slot_idx[b];
            const float ry = (y[u] + y[dd]) - (yh + yh);
            const float rz = (z[u] + z[dd]) - (zh + zh);
            const float score = ry * ry + rz * rz;
            if (!(score <= cut2)) continue;
            if (bu < 0 || score < best || (score == best && (u < bu || (u == bu && dd < bd)))) {
              best = score;
              bu = u;
              bd = dd;
            }
          }
        }
        if (bu >= 0) {
          up_raw[h] = bu;
          down_raw[h] = bd;
          break;
        }
      }
    }
    // O5: keep mutual links only, evaluated from the raw arrays
    up.assign(n, -1);
    down.assign(n, -1);
    for (int32_t h = 0; h < n; ++h) {
      if (up_raw[h] >= 0 && down_raw[up_raw[h]] == h) up[h] = up_raw[h];
      if (down_raw[h] >= 0 && up_raw[down_raw[h]] == h) down[h] = down_raw[h];
    }
  }

  // -------- O6 + O7: starts, tracklet construction, hit weights
  void construct_tracklets() {
    starts.clear();
    for (int32_t h = 0; h < n; ++h)
      if (down[h] < 0 && up[h] >= 0 && up[up[h]] >= 0) starts.push_back(h);
    tracklets.assign(starts.size(), Tracklet());
    hitw.assign(n, 0);
    const float cb = curvature_factor<float>(p);
    const float vy = p.sigma_y * p.sigma_y, vz = p.sigma_z * p.sigma_z;
    for (size_t id = 0; id < starts.size(); ++id) {
      Tracklet& t = tracklets[id];
      t.start = starts[id];
      build_tracklet(t, cb, vy, vz);
      t.n = (int32_t)t.hits.size();
      t.valid = t.n >= p.min_hits;
      if (t.valid) {
        const uint64_t key = ((uint64_t)t.n << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)id);
        for (int32_t h : t.hits) hitw[h] = std::max(hitw[h], key);
      }
    }
  }

  // The chain of a start h: h, up[h], up[up[h]], ...  A chain's innermost cluster has no
  // lower neighbour, so it never gets an up link of its own; it is recovered as the
  // start's raw down neighbour d when d has no up link (d is then prepended).
  int32_t chain_first(int32_t h) const {
    const int32_t d = down_raw[h];
    return (d >= 0 && up_raw[d] < 0) ? d : h;
  }
  int32_t chain_next(int32_t c, int32_t h, int32_t first) const {
    return (c == first && first != h) ? h : up[c];
  }

  void build_tracklet(Tracklet& t, float cb, float vy, float vz) {
    const int32_t c0 = chain_first(t.start);
    const int32_t c1 = chain_next(c0, t.start, c0), c2 = chain_next(c1, t.start, c0);
    const int s = sector[c0], j = job_of[c0];
    float P[5], L[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, C[15];
    const float dx2 = kGeo.x[row[c2]] - kGeo.x[row[c0]];
    const float dy2 = y[c2] - y[c0];
    const float dz2 = z[c2] - z[c0];
    const float den = std::sqrt(dx2 * dx2 + dy2 * dy2);
    P[0] = y[c0];
    P[1] = z[c0];
    P[2] = dy2 / den;
    P[3] = dz2 / den;
    P[4] = 0.f;
    for (int i = 0; i < 15; ++i) C[i] = 0.f;
    C[tri(0, 0)] = p.cy0; C[tri(1, 1)] = p.cz0; C[tri(2, 2)] = p.cs0;
    C[tri(3, 3)] = p.ct0; C[tri(4, 4)] = p.ck0;
    float x = kGeo.x[row[c0]];
    auto keep_state = [&]() {
      std::memcpy(t.P, P, sizeof(P));
      std::memcpy(t.C, C, sizeof(C));
      t.x = x;
    };
    keep_state();  // the recorded state is the initial one until a cluster is accepted
    // the chain: every chain cluster is used unconditionally
    for (int32_t h = c0; h >= 0; h = chain_next(h, t.start, c0)) {
      const float xh = kGeo.x[row[h]];
      if (!propagate(P, L, C, x, xh, cb, p.smax)) return;
      x = xh;
      if (!kf_update(P, L, C, y[h], z[h], vy, vz, p.smax, (float*)nullptr)) return;
      t.hits.push_back(h);
      keep_state();
    }
    // following on the rows above the chain
    int misses = 0;
    for (int r = row[t.hits.back()] + 1; r < kRows; ++r) {
      const float xr = kGeo.x[r];
      if (!propagate(P, L, C, x, xr, cb, p.smax)) return;
      x = xr;
      const SInv<float> si = s_inverse(C, vy, vz);
      if (!si.ok) return;
      const float wy = p.nwin * std::sqrt(C[tri(0, 0)] + vy);
      const float wz = p.nwin * std::sqrt(C[tri(1, 1)] + vz);
      int64_t lo, hi;
      z_range(slot(j, s, r), P[1] - wz - 0.01f, P[1] + wz + 0.01f, lo, hi);
      int32_t best = -1;
      float bchi = 0.f;
      for (int64_t a = lo; a < hi; ++a) {
        const int32_t c = slot_idx[a];
        const float r0 = (y[c] - P[0]) - L[0];
        const float r1 = (z[c] - P[1]) - L[1];
        if (!(std::fabs(r0) <= wy) || !(std::fabs(r1) <= wz)) continue;
        const float chi2 = chi2_of(si, r0, r1);
        if (best < 0 || chi2 < bchi || (chi2 == bchi && c < best)) {
          best = c;
          bchi = chi2;
        }
      }
      if (best >= 0 && bchi <= p.chi2_follow) {
        if (!kf_update(P, L, C, y[best], z[best], vy, vz, p.smax, (float*)nullptr)) return;
        t.hits.push_back(best);
        keep_state();
        misses = 0;
      } else if (++misses >= p.max_miss) {
        return;
      }
    }
  }

  // -------- O9: selection
  void select_tracks() {
    tracks.clear();
    for (size_t id = 0; id < tracklets.size(); ++id) {
      const Tracklet& t = tracklets[id];
      if (!t.valid) continue;
      const uint64_t key = ((uint64_t)t.n << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)id);
      Track tr;
      for (int32_t h : t.hits)
        if (hitw[h] == key) tr.hits.push_back(h);
      if ((int32_t)tr.hits.size() < p.min_hits) continue;
      tr.tracklet = (int32_t)id;
      tr.job = job_of[t.start];
      tr.sector = sector[t.start];
      tr.event = job_event[tr.job];
      tracks.push_back(std::move(tr));
    }
  }

  // -------- O9: Kalman refit from the outermost to the innermost hit
  template <class T>
  bool fit(const std::vector<int32_t>& hits, const float* sinit, int sec_outer,
           const std::vector<int>& hit_sector, T* P, T* C, T& xout, T& chi2, int32_t& ndf,
           T* Lout = nullptr, const std::vector<float>* zshift = nullptr) {
    const T cb = curvature_factor<T>(p);
    const T vy = (T)p.sigma_y * (T)p.sigma_y, vz = (T)p.sigma_z * (T)p.sigma_z;
    const T smax = (T)p.smax;
    const int nh = (int)hits.size();
    const int32_t ho = hits[nh - 1];
    P[0] = (T)y[ho];
    P[1] = (T)z[ho];
    P[2] = (T)sinit[0];
    P[3] = (T)sinit[1];
    P[4] = (T)sinit[2];
    T L[5] = {T(0), T(0), T(0), T(0), T(0)};
    for (int i = 0; i < 15; ++i) C[i] = T(0);
    C[tri(0, 0)] = (T)p.cy1; C[tri(1, 1)] = (T)p.cz1; C[tri(2, 2)] = (T)p.cs1;
    C[tri(3, 3)] = (T)p.ct1; C[tri(4, 4)] = (T)p.ck1;
    T x = (T)kGeo.x[row[ho]];
    chi2 = T(0);
    int cur_sec = sec_outer;
    for (int i = nh - 1; i >= 0; --i) {
      const int32_t h = hits[i];
      if (hit_sector[i] != cur_sec) {
        if ((hit_sector[i] < kRowsPerSide) != (cur_sec < kRowsPerSide)) {
          // crossing the central membrane into the inner piece's side (A21): the same
          // sector frame, z moved by the drift of the link's collision time
          acc(P[1], L[1], zshift ? (T)(*zshift)[i] : T(0));
        } else {
          // crossing into the neighbouring sector of the inner piece (O10)
          if (!rotate(P, L, C, x, cur_sec, hit_sector[i])) return false;
        }
        cur_sec = hit_sector[i];
      }
      const T xh = (T)kGeo.x[row[h]];
      if (!propagate(P, L, C, x, xh, cb, smax)) return false;
      x = xh;
      T c2;
      if (!kf_update(P, L, C, (T)y[h], (T)z[h], vy, vz, smax, &c2)) return false;
      chi2 = chi2 + c2;
    }
    xout = x;
    ndf = 2 * nh - 5;
    if (Lout)
      for (int i = 0; i < 5; ++i) Lout[i] = L[i];
    return true;
  }

  template <class T> bool rotate(T* P, T* L, T* C, T& x, int from, int to) {
    return rotate_sector(P, L, C, x, from, to, curvature_factor<T>(p), (T)p.smax);
  }

  void fit_all() {
    for (Track& tr : tracks) fit_track(tr);
    if (p.ext_down) extend_down();
  }

  // -------- A13: downward extension of the selected tracks.  The chain of a track need not
  // start at the track's first row (a cluster lost to inefficiency or a link lost to a
  // denser neighbourhood breaks it), and the following only visits the rows above the chain.
  // So every track whose fit succeeded continues below its innermost hit: from the FP32
  // fitted state there (compensation terms included) the rows under it are visited one by
  // one, inwards, in the track's sector, the way the following visits the rows above a
  // chain (O7: transport, 3-sigma window, minimum chi2 with ties to the smaller index, the
  // chi2 cut, at most max_miss consecutive misses), except that only clusters owned by no
  // selected track may be taken.  Two tracks may take the same cluster: it goes to the track
  // with more owned hits, then to the smaller track id, and a track keeps its extension hits
  // up to the first one it lost.  The kept hits are put in front of the track's hits (rows
  // ascending) and the track is fitted again over the whole list.
  void extend_down() {
    const float cb = curvature_factor<float>(p);
    const float vy = p.sigma_y * p.sigma_y, vz = p.sigma_z * p.sigma_z;
    const int K = (int)tracks.size();
    std::vector<uint8_t> owned(n, 0);
    for (const Track& tr : tracks)
      for (int32_t h : tr.hits) owned[h] = 1;
    std::vector<std::vector<int32_t>> found(K);
    for (int k = 0; k < K; ++k) {
      const Track& tr = tracks[k];
      if (tr.ndf < 0) continue;
      float P[5], L[5], C[15];
      std::memcpy(P, tr.P, sizeof(P));
      std::memcpy(L, tr.L, sizeof(L));
      std::memcpy(C, tr.C, sizeof(C));
      float x = tr.x;
      int misses = 0;
      for (int r = row[tr.hits.front()] - 1; r >= 0; --r) {
        const float xr = kGeo.x[r];
        if (!propagate(P, L, C, x, xr, cb, p.smax)) break;
        x = xr;
        const SInv<float> si = s_inverse(C, vy, vz);
        if (!si.ok) break;
        const float wy = p.nwin * std::sqrt(C[tri(0, 0)] + vy);
        const float wz = p.nwin * std::sqrt(C[tri(1, 1)] + vz);
        int64_t lo, hi;
        z_range(slot(tr.job, tr.sector, r), P[1] - wz - 0.01f, P[1] + wz + 0.01f, lo, hi);
        int32_t best = -1;
        float bchi = 0.f;
        for (int64_t a = lo; a < hi; ++a) {
          const int32_t c = slot_idx[a];
          if (owned[c]) continue;
          const float r0 = (y[c] - P[0]) - L[0];
          const float r1 = (z[c] - P[1]) - L[1];
          if (!(std::fabs(r0) <= wy) || !(std::fabs(r1) <= wz)) continue;
          const float chi2 = chi2_of(si, r0, r1);
          if (best < 0 || chi2 < bchi || (chi2 == bchi && c < best)) {
            best = c;
            bchi = chi2;
          }
        }
        if (best >= 0 && bchi <= p.chi2_follow) {
          if (!kf_update(P, L, C, y[best], z[best], vy, vz, p.smax, (float*)nullptr)) break;
          found[k].push_back(best);
          misses = 0;
        } else if (++misses >= p.max_miss) {
          break;
        }
      }
    }
    // contested clusters: more owned hits first, then the smaller track id
    std::vector<uint64_t> key(K);
    for (int k = 0; k < K; ++k)
      key[k] = ((uint64_t)tracks[k].hits.size() << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
    std::vector<uint64_t> claim(n, 0);
    for (int k = 0; k < K; ++k)
      for (int32_t c : found[k]) claim[c] = std::max(claim[c], key[k]);
    for (int k = 0; k < K; ++k) {
      size_t m = 0;
      while (m < found[k].size() && claim[found[k][m]] == key[k]) ++m;
      if (m == 0) continue;
      Track& tr = tracks[k];
      std::vector<int32_t> h(found[k].rend() - (std::ptrdiff_t)m, found[k].rend());  // rows ascending
      h.insert(h.end(), tr.hits.begin(), tr.hits.end());
      tr.hits.swap(h);
      tr.n_ext = (int32_t)m;
      fit_track(tr);
    }
  }

  void fit_track(Track& tr) {
    std::vector<int> hs(tr.hits.size());
    for (size_t i = 0; i < tr.hits.size(); ++i) hs[i] = sector[tr.hits[i]];
    const int self = (int)(&tr - tracks.data());
    const int last = tr.pieces.empty() ? self : tr.pieces.back();
    const Tracklet& st = tracklets[tracks[last].tracklet];
    const float sinit[3] = {st.P[2], st.P[3], st.P[4]};
    const int so = hs.back();
    // A21: the z shift at each membrane crossing of a chain, entered on the inner piece's
    // outermost hit: the drift of the link's collision time, twice (one side's z is short
    // of the true z by v t0, the other's long by as much)
    std::vector<float> zs(tr.hits.size(), 0.f);
    if (!tr.pieces.empty()) {
      std::vector<int> chain = {self};
      chain.insert(chain.end(), tr.pieces.begin(), tr.pieces.end());
      size_t absorbed = 0;
      for (size_t c = 1; c < chain.size(); ++c) absorbed += tracks[chain[c]].hits.size();
      size_t pos = tr.hits.size() - absorbed;  // one past the head's own hits
      for (size_t c = 0; c + 1 < chain.size(); ++c) {
        const int inner = chain[c];
        const bool a_side = tracks[inner].sector < kRowsPerSide;
        if (a_side != (tracks[chain[c + 1]].sector < kRowsPerSide)) {
          const float d = (2.0f * p.v_drift) * tracks[inner].link_t0;
          zs[pos - 1] = a_side ? -d : d;
        }
        pos += tracks[chain[c + 1]].hits.size();
      }
    }
    if (!fit<float>(tr.hits, sinit, so, hs, tr.P, tr.C, tr.x, tr.chi2, tr.ndf, tr.L, &zs)) {
      tr.ndf = -1;
      for (float& v : tr.P) v = NAN;
    }
    const auto t0 = std::chrono::steady_clock::now();
    if (!fit<double>(tr.hits, sinit, so, hs, tr.Pd, tr.Cd, tr.xd, tr.chi2d, tr.ndfd, nullptr, &zs)) {
      tr.ndfd = -1;
      for (double& v : tr.Pd) v = NAN;
    }
    fp64_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // -------- O10: merge track pieces that continue into an adjacent sector (same side).
  // A (inner piece) ends within merge_edge of the sector edge it is heading for; B (outer
  // piece) lies in the adjacent sector and starts within merge_edge of the same edge.
  // A's tracklet end state is rotated into B's frame, propagated to B's innermost plane
  // and compared with B's fitted state: chi2 = d^T (C_A + C_B)^-1 d.  Pairs with
  // chi2 <= chi2_merge that are each other's best (ties: smaller id) are joined; joins
  // chain through several sectors.  Merged hit list: inner piece first.  The merged
  // track keeps the innermost piece's id and is refitted across the sector crossings.
  void merge() {
    const float cb = curvature_factor<float>(p);
    const int K = (int)tracks.size();
    std::vector<float> bestA(K, 0.f), bestB(K, 0.f);
    std::vector<int32_t> argA(K, -1), argB(K, -1);
    // the tracks of each (event, sector), in ascending id: the only B a given A can pair with
    std::unordered_map<int64_t, std::vector<int32_t>> by_sector;
    for (int b = 0; b < K; ++b) by_sector[(int64_t)tracks[b].event * kSectors + tracks[b].sector].push_back(b);
    const std::vector<int32_t> none;
    auto consider = [&](int a, int b, float c) {
      if (argA[a] < 0 || c < bestA[a] || (c == bestA[a] && b < argA[a])) { bestA[a] = c; argA[a] = b; }
      if (argB[b] < 0 || c < bestB[b] || (c == bestB[b] && a < argB[b])) { bestB[b] = c; argB[b] = a; }
    };
    for (int a = 0; a < K; ++a) {
      const Track& A = tracks[a];
      if (A.ndf < 0) continue;
      const Tracklet& ta = tracklets[A.tracklet];
      if (p.merge_membrane) membrane_candidates(a, by_sector, consider);
      const float edge = ta.x * kGeo.tan10 - std::fabs(ta.P[0]);
      if (!(edge <= p.merge_edge)) continue;
      const int dir = ta.P[0] > 0.f ? 1 : kRowsPerSide - 1;
      const int sb = (A.sector / kRowsPerSide) * kRowsPerSide + (A.sector % kRowsPerSide + dir) % kRowsPerSide;
      const auto it = by_sector.find((int64_t)A.event * kSectors + sb);
      for (const int b : it == by_sector.end() ? none : it->second) {
        const Track& B = tracks[b];
        if (B.ndf < 0 || B.event != A.event || B.sector != sb) continue;
        const int32_t hb = B.hits.front();
        const float eb = kGeo.x[row[hb]] * kGeo.tan10 - std::fabs(y[hb]);
        if (!(eb <= p.merge_edge)) continue;
        // B starts at the edge it shares with A's sector: its -y edge when A leaves
        // through its +y edge, and the other way round
        if (dir == 1 ? !(y[hb] < 0.f) : !(y[hb] >= 0.f)) continue;
        if (!(std::fabs(ta.P[1] - z[hb]) <= p.merge_dz)) continue;
        float P[5], L[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, C[15];
        std::memcpy(P, ta.P, sizeof(P));
        std::memcpy(C, ta.C, sizeof(C));
        float x = ta.x;
        if (!rotate(P, L, C, x, A.sector, sb)) continue;
        if (!propagate(P, L, C, x, B.x, cb, p.smax)) continue;
        const float c = merge_chi2(P, C, B.P, B.C);
        if (!(c <= p.chi2_merge)) continue;
        consider(a, b, c);
      }
    }
    std::vector<int32_t> prev(K, -1);
    for (int a = 0; a < K; ++a) {
      const int b = argA[a];
      if (b >= 0 && argB[b] == a) {
        tracks[a].partner = b;
        prev[b] = a;
        if ((tracks[a].sector < kRowsPerSide) != (tracks[b].sector < kRowsPerSide)) {
          float P[5], C[15];
          membrane_transport(tracklets[tracks[a].tracklet], tracks[b], P, C);
          tracks[a].link_t0 = membrane_t0(tracks[a].sector < kRowsPerSide, P[1], tracks[b].P[1]);
        }
      }
    }
    for (int a = 0; a < K; ++a) {
      if (prev[a] >= 0 || tracks[a].partner < 0) continue;   // chain heads only
      Track& A = tracks[a];
      // a chain walked from its head is a simple path (every piece has one inner partner)
      int inner = a;
      for (int b = A.partner; b >= 0 && (int)A.pieces.size() < kRowsPerSide; b = tracks[b].partner) {
        tracks[b].merged_into = a;
        A.pieces.push_back(b);
        A.hits.insert(A.hits.end(), tracks[b].hits.begin(), tracks[b].hits.end());
        A.sector2 = tracks[b].sector;
        // the chain's collision time: its innermost membrane link's (A21)
        if (std::isnan(A.t0m) && (tracks[inner].sector < kRowsPerSide) != (tracks[b].sector < kRowsPerSide))
          A.t0m = tracks[inner].link_t0;
        inner = b;
      }
      fit_track(A);
    }
  }

  // -------- A21: merge across the central membrane.  A track from a vertex off z = 0 whose
  // z changes sign inside the chamber leaves a piece on each side, in the same sector frame.
  // In a time frame the two sides' measured z are off by v t0 in opposite directions (side
  // A: z - v t0, side C: z + v t0), so z cannot be compared; the other four parameters can.
  // A (inner piece) heads for the membrane: tan lambda < 0 on side A, > 0 on side C.  B
  // lies in the same sector on the other side of the same event, starts beyond A's end
  // (B.x > A's end x), has the same sign of tan lambda, and its innermost measured z
  // mirrors A's end: |z_A + z_B| <= merge_dz (both ends at the membrane, so the true z of
  // both are near 0 and the offsets cancel in the sum).  A's tracklet end state is carried
  // to B's innermost plane; the true z there, the mean of the two measured z, must be
  // within merge_edge of the membrane, and chi2 = d^T (C_A + C_B)^-1 d over (y, sin phi,
  // tan lambda, q/pT) <= chi2_merge.  These candidates join the sector candidates in the
  // mutual-best pairing.  The link's collision time is (z_B - z_A) / (2 v) with A on side A
  // (the other way round on side C).
  bool membrane_transport(const Tracklet& ta, const Track& B, float* P, float* C) const {
    float L[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    std::memcpy(P, ta.P, sizeof(float) * 5);
    std::memcpy(C, ta.C, sizeof(float) * 15);
    float x = ta.x;
    return propagate(P, L, C, x, B.x, curvature_factor<float>(p), p.smax);
  }
  float membrane_t0(bool a_side, float za, float zb) const {
    return a_side ? (zb - za) / (2.0f * p.v_drift) : (za - zb) / (2.0f * p.v_drift);
  }
  template <class F>
  void membrane_candidates(int a, const std::unordered_map<int64_t, std::vector<int32_t>>& by_sector,
                           F&& consider) {
    const Track& A = tracks[a];
    const Tracklet& ta = tracklets[A.tracklet];
    const bool a_side = A.sector < kRowsPerSide;
    if (!(a_side ? ta.P[3] < 0.f : ta.P[3] > 0.f)) return;
    const int sb = (A.sector + kRowsPerSide) % kSectors;
    const auto it = by_sector.find((int64_t)A.event * kSectors + sb);
    if (it == by_sector.end()) return;
    for (const int b : it->second) {
      const Track& B = tracks[b];
      if (B.ndf < 0 || B.event != A.event || B.sector != sb) continue;
      if (!(a_side ? B.P[3] < 0.f : B.P[3] > 0.f)) continue;
      if (!(B.x > ta.x)) continue;
      if (!(std::fabs(ta.P[1] + z[B.hits.front()]) <= p.merge_dz)) continue;
      float P[5], C[15];
      if (!membrane_transport(ta, B, P, C)) continue;
      if (!(std::fabs((P[1] + B.P[1]) * 0.5f) <= p.merge_edge)) continue;
      const float c = membrane_chi2(P, C, B.P, B.C);
      if (!(c <= p.chi2_merge)) continue;
      consider(a, b, c);
    }
  }

  // chi2 = d^T (CA + CB)^-1 d over y, sin phi, tan lambda and q/pT (indices 0, 2, 3, 4), by
  // Cholesky in fixed order
  static float membrane_chi2(const float* PA, const float* CA, const float* PB, const float* CB) {
    const int ix[4] = {0, 2, 3, 4};
    float S[10], d[4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j <= i; ++j) S[tri(i, j)] = CA[tri(ix[i], ix[j])] + CB[tri(ix[i], ix[j])];
    for (int i = 0; i < 4; ++i) d[i] = PA[ix[i]] - PB[ix[i]];
    float L[10];
    for (int i = 0; i < 4; ++i) {
      for (int j = 0; j <= i; ++j) {
        float acc_ = S[tri(i, j)];
        for (int k = 0; k < j; ++k) acc_ = acc_ - L[tri(i, k)] * L[tri(j, k)];
        if (i == j) {
          if (!(acc_ > 0.f)) return INFINITY;
          L[tri(i, i)] = std::sqrt(acc_);
        } else {
          L[tri(i, j)] = acc_ / L[tri(j, j)];
        }
      }
    }
    float w[4];
    float c = 0.f;
    for (int i = 0; i < 4; ++i) {
      float acc_ = d[i];
      for (int k = 0; k < i; ++k) acc_ = acc_ - L[tri(i, k)] * w[k];
      w[i] = acc_ / L[tri(i, i)];
      c = c + w[i] * w[i];
    }
    return c;
  }

  // chi2 = d^T (CA + CB)^-1 d over the 5 parameters, by Cholesky in fixed order
  static float merge_chi2(const float* PA, const float* CA, const float* PB, const float* CB) {
    float S[15], d[5];
    for (int i = 0; i < 15; ++i) S[i] = CA[i] + CB[i];
    for (int i = 0; i < 5; ++i) d[i] = PA[i] - PB[i];
    float L[15];
    for (int i = 0; i < 5; ++i) {
      for (int j = 0; j <= i; ++j) {
        float acc = S[tri(i, j)];
        for (int k = 0; k < j; ++k) acc = acc - L[tri(i, k)] * L[tri(j, k)];
        if (i == j) {
          if (!(acc > 0.f)) return INFINITY;
          L[tri(i, i)] = std::sqrt(acc);
        } else {
          L[tri(i, j)] = acc / L[tri(j, j)];
        }
      }
    }
    float w[5];
    float c = 0.f;
    for (int i = 0; i < 5; ++i) {
      float acc = d[i];
      for (int k = 0; k < i; ++k) acc = acc - L[tri(i, k)] * w[k];
      w[i] = acc / L[tri(i, i)];
      c = c + w[i] * w[i];
    }
    return c;
  }
};

// ---------------------------------------------------------------- C: track-model compression
// Section 5: the clusters are stored as residuals to the fitted tracks instead of as
// absolute coordinates, so that the entropy coder that follows sees small numbers.
// The paper gives no format; the reading written out here (C1-C5):
//  C1 The prediction for a cluster of track i at (sector s, row r) starts from the
//     fitted state (y, z, sin phi, tan lambda, q/pT) at x_ref in the frame of the
//     track's sector, turns it one sector at a time towards s (O10 rotation, state
//     only, on the same side of the membrane, the shorter way round), then transports
//     it to the plane x_r (O2, state only).  There is no prediction when the fit
//     failed (ndf < 0), the sides differ, or a rotation or the transport fails.
//  C2 With a prediction (py, pz) the codes are e = rint((v - p) * (1/q)) per coordinate,
//     in FP32; if |e| > 32767 for either coordinate, or without prediction, the cluster
//     takes absolute codes e = rint(v * (1/q)) and the flag "absolute".
//  C3 Absolute codes saturate at +-32767 and raise the range status; an invalid cluster
//     (sector >= 36, row outside 0..151, non-finite y or z, or a hit index outside the
//     cluster list) is written as the record 0x7FFF with zero codes and raises it too.
//  C4 Stream order: the hits of every track in track order, then every cluster that is
//     in no track, in input order, with absolute codes.
//  C5 Decoding: v = p + e*q for residual codes, v = e*q for absolute ones (FP32, each
//     operation rounded once); the record gives sector and row.
//  C7 Time frames: the drift-shifted z of a continuous read-out spans thousands of cm
//     (+-2580 cm in a 1 ms frame), beyond 16-bit codes at q = 1/32 cm.  With a high-byte
//     field, an absolute z code takes 24 bits: e = rint(z * (1/q)) saturated at
//     +-(2^23 - 1), stored as its low 16 bits (ez) and the signed high byte (ez_hi), so
//     that e = ez_hi * 2^16 + (ez as unsigned); residual and invalid records have
//     ez_hi = 0.  Absolute y codes keep 16 bits (|y| <= 43.2 cm).
// The record of a cluster: rs = row | sector << 8 | absolute << 15, plus the two codes.
constexpr uint16_t kRecInvalid = 0x7FFF;
constexpr int kCodeMax = 32767;

// C1, rotation step: the state part of O10 (rotate() above without the covariance).
bool rotate_state(const Params& p, float* P, float& x, int from, int to) {
  if (from / kRowsPerSide != to / kRowsPerSide) return false;
  const int df = ((to % kRowsPerSide) - (from % kRowsPerSide) + kRowsPerSide) % kRowsPerSide;
  if (df != 1 && df != kRowsPerSide - 1) return false;
  const float ca = kGeo.cos20;
  const float sa = df == 1 ? kGeo.sin20 : -kGeo.sin20;
  const float s = P[2];
  const float c = std::sqrt((1.f - s) * (1.f + s));
  const float xn = x * ca + P[0] * sa;
  const float yn = P[0] * ca - x * sa;
  const float sn = s * ca - c * sa;
  const float cn = c * ca + s * sa;
  if (!(cn > 0.f) || !(std::fabs(sn) < p.smax)) return false;
  P[0] = yn;
  P[2] = sn;
  x = xn;
  for (int i = 0; i < 5; ++i)
    if (!(P[i] - P[i] == 0.f)) return false;
  return true;
}

// C1, transport: the state part of O2 (propagate() above without Jacobian and covariance).
template <class T> bool transport_state(const Params& p, T* P, T x1, T x2) {
  const T dx = x2 - x1;
  if (dx == T(0)) return true;
  const T curv = P[4] * curvature_factor<T>(p);
  const T s1 = P[2];
  const T s2 = s1 + curv * dx;
  if (!(std::fabs(s2) < (T)p.smax)) return false;
  const T c1 = std::sqrt((T(1) - s1) * (T(1) + s1));
  const T c2 = std::sqrt((T(1) - s2) * (T(1) + s2));
  const T f = (s1 + s2) / (c1 + c2);
  const T dy = dx * f;
  T ch = std::sqrt(dx * dx + dy * dy);
  if (dx < T(0)) ch = -ch;
  const T u = curv * ch * T(0.5);
  if (!(std::fabs(u) < T(1))) return false;
  T A, B;
  asinc(u, A, B);
  P[0] = P[0] + dy;
  P[1] = P[1] + P[3] * (ch * A);
  P[2] = P[2] + curv * dx;
  return true;
}

//  T1 Collision time of a track in continuous read-out.  A cluster's measured z is the
//     drift distance recomputed from its arrival time, so a collision at time t0 after
//     the frame start shows every cluster shifted by v_d t0 towards the central membrane's
//     far side: z_meas = z - v_d t0 on side A, z + v_d t0 on side C.  A primary comes from
//     the nominal vertex on the beam line (z = 0), which is the plane x = 0 of its
//     sector frame; there the fitted helix has z_meas = -v_d t0 (A) or +v_d t0 (C).  So
//     the fitted state is transported (O2, state alone) from its reference plane to
//     x = 0 and t0 = -z/v_d on side A, +z/v_d on side C.  NaN when the fit failed or the
//     transport fails (|sin phi| >= smax on the way).
template <class T> T collision_time(const Params& p, const T* Pfit, T xref, int sector) {
  T P[5];
  for (int i = 0; i < 5; ++i) P[i] = Pfit[i];
  if (!transport_state(p, P, xref, T(0))) return (T)NAN;
  const T z0 = P[1];
  return (sector < kRowsPerSide ? -z0 : z0) / (T)p.v_drift;
}

// C1: the predicted (y, z) of a cluster at (sec, row) of a track with fitted state Pfit.
bool predict(const Params& p, const float* Pfit, float xref, int sref, int sec, int row, float& py,
             float& pz) {
  if (sref < 0 || sref >= kSectors || sec / kRowsPerSide != sref / kRowsPerSide) return false;
  float P[5];
  for (int i = 0; i < 5; ++i) P[i] = Pfit[i];
  float x = xref;
  const int steps = ((sec % kRowsPerSide) - (sref % kRowsPerSide) + kRowsPerSide) % kRowsPerSide;
  const int dir = steps <= kRowsPerSide / 2 ? 1 : -1;
  const int nst = dir == 1 ? steps : kRowsPerSide - steps;
  int cur = sref;
  for (int k = 0; k < nst; ++k) {
    const int nxt = (cur / kRowsPerSide) * kRowsPerSide + (cur % kRowsPerSide + dir + kRowsPerSide) % kRowsPerSide;
    if (!rotate_state(p, P, x, cur, nxt)) return false;
    cur = nxt;
  }
  if (!transport_state(p, P, x, kGeo.x[row])) return false;
  py = P[0];
  pz = P[1];
  return true;
}

bool cluster_ok(uint8_t sec, int16_t row, float y, float z) {
  return sec < kSectors && row >= 0 && row < kRows && y - y == 0.f && z - z == 0.f;
}

// C3: absolute code with saturation.
int16_t abs_code(float v, float iq, int32_t& status) {
  float e = std::rint(v * iq);
  if (e > (float)kCodeMax) { e = (float)kCodeMax; status |= 1; }
  if (e < -(float)kCodeMax) { e = -(float)kCodeMax; status |= 1; }
  return (int16_t)e;
}

// C7: 24-bit absolute code, split into the low 16 bits and the signed high byte.
constexpr int32_t kWideMax = (1 << 23) - 1;
void abs_code_wide(float v, float iq, int16_t& lo, int8_t& hi, int32_t& status) {
  float e = std::rint(v * iq);
  if (e > (float)kWideMax) { e = (float)kWideMax; status |= 1; }
  if (e < -(float)kWideMax) { e = -(float)kWideMax; status |= 1; }
  const int32_t c = (int32_t)e;
  lo = (int16_t)(uint16_t)(c & 0xFFFF);
  hi = (int8_t)(c >> 16);
}

struct TrackHeaders {
  int32_t K;
  const int32_t* off;
  const float* param;
  const float* x_ref;
  const int32_t* sector;
  const int32_t* ndf;
};

// ---------------------------------------------------------------- E: entropy coding (rANS)
// Section 5: every detector's data, the TPC's after the track-model compression, goes
// through a common rANS entropy coder (Table 1: TPC rANS encoding; Table 2: decoding).  The
// paper names the coder only; the reading (E1-E5) is static range ANS as Duda defined it:
//  E1 One model per stream of 16-bit symbols: counts c_s over the stream, K = symbols that
//     occur, M = 2^16; f_s = max(1, floor(c_s (M - K) / n)) for those, 0 for the others;
//     the remainder M - sum f goes to the most frequent symbol (ties: the smaller symbol).
//     C_s = sum of f_t over t < s.
//  E2 Coder: 32-bit state x in [2^16, 2^32), 16-bit words.  Encoding s: if x >= f_s 2^16,
//     emit x mod 2^16 and x <- floor(x / 2^16); then x <- floor(x / f_s) 2^16 +
//     (x mod f_s) + C_s.  The state starts at 2^16.
//  E3 Decoding: slot = x mod 2^16, s the symbol with C_s <= slot < C_s + f_s,
//     x <- f_s floor(x / 2^16) + slot - C_s, and if x < 2^16, x <- x 2^16 + next word.
//  E4 Lanes: the stream is cut into chunks of 64 S symbols (S = 512); lane l of chunk k
//     codes the symbols k 64 S + l + 64 m that exist, with its own state, last symbol
//     first, so that its decoder reads them first to last.  A lane's words in decoding
//     order: the final state (high word, low word), then the emitted words, last emitted
//     first.  A lane without symbols has no words.
//  E5 The lanes' words are concatenated in lane order; lane_off[l] is the offset of lane l.
constexpr int kRansLaneSymbols = 512;
constexpr int kRansLanesPerChunk = 64;
constexpr uint32_t kRansM = 1u << 16;
constexpr uint32_t kRansL = 1u << 16;

int64_t rans_lanes(int64_t n) {
  const int64_t chunk = (int64_t)kRansLanesPerChunk * kRansLaneSymbols;
  return (n + chunk - 1) / chunk * kRansLanesPerChunk;
}
// symbols of lane l (chunk l / 64, lane l % 64): indices first + 64 m, m < count
void rans_lane(int64_t n, int64_t l, int64_t& first, int64_t& count) {
  const int64_t k = l / kRansLanesPerChunk, j = l % kRansLanesPerChunk;
  first = k * kRansLanesPerChunk * kRansLaneSymbols + j;
  count = first < n ? std::min<int64_t>(kRansLaneSymbols, (n - first + kRansLanesPerChunk - 1) / kRansLanesPerChunk) : 0;
}

// ---------------------------------------------------------------- F: cluster finding
// Section 5: the TPC clusters are found on the GPUs from the zero-suppressed digits, before
// the tracking.  The paper gives neither the pad plane nor the finder; the reading (F1-F6):
//  F1 Pad plane: row r holds P_r = 2 ceil(x_r tan 10 deg / pitch) pads (x_r in double),
//     pad p centred at y = (p + 1/2) pitch - P_r pitch / 2; time bins of `bin` cm of |z|,
//     bin t centred at |z| = (t + 1/2) bin, t < n_time.
//  F2 Charge map: each cell (sector, row, pad, time) holds the sum of the ADC counts of the
//     digits in it; digits outside the sector/row/pad/time ranges are dropped and raise the
//     range status.
//  F3 Peak: a digit whose cell charge q >= q_min and, over the 8 neighbouring cells of its
//     row (cells outside the pad or time range count as 0), q > q_n for the neighbours that
//     come before it in (pad, time) order and q >= q_n for those after (so of two equal
//     neighbouring maxima the earlier one is the peak).
//  F4 Cluster of a peak at (p, t): over its 3 x 3 cells, Q = sum q, S_p = sum q dp,
//     S_t = sum q dt, S_pp = sum q dp^2, S_tt = sum q dt^2 (integers, exact); in FP32
//     pad = p + S_p / Q, time = t + S_t / Q, sigma_pad = sqrt(max(0, S_pp / Q - (S_p / Q)^2))
//     (q_min >= 1, so Q > 0)
//     and likewise in time; y = (pad + 1/2) pitch - P_r pitch / 2 (the last term rounded
//     once from double), z = (time + 1/2) bin, negative on side C; q_max = the peak's q.
//  F5 Clusters come in the order of their peak digits in the input.
//  F6 Duplicated digits add up in the map; each copy of a peak digit reports the cluster.
int32_t cf_pads(int r, float pitch) {
  const double x = 85.0 + (double)r * 160.0 / 151.0;
  return 2 * (int32_t)std::ceil(x * std::tan(10.0 * 3.14159265358979323846 / 180.0) / (double)pitch);
}

}  // namespace

// ============================================================== C interface (ctypes)
extern "C" {

void* orc_create(int32_t n, const uint8_t* sector, const int16_t* row, const float* y,
                 const float* z, int32_t n_jobs, const int32_t* job_off, const int32_t* job_event,
                 const Params* p) {
  Oracle* o = new Oracle();
  o->p = *p;
  o->n = n;
  o->J = n_jobs;
  o->sector.assign(sector, sector + n);
  o->row.assign(row, row + n);
  o->y.assign(y, y + n);
  o->z.assign(z, z + n);
  o->job_off.assign(job_off, job_off + n_jobs + 1);
  o->job_of.assign(n, 0);
  o->job_event.resize(n_jobs);
  for (int j = 0; j < n_jobs; ++j) o->job_event[j] = job_event ? job_event[j] : j;
  o->valid.assign(n, 1);
  for (int j = 0; j < n_jobs; ++j)
    for (int32_t i = job_off[j]; i < job_off[j + 1]; ++i) o->job_of[i] = j;
  for (int32_t i = 0; i < n; ++i) {
    const bool ok = sector[i] < kSectors && row[i] >= 0 && row[i] < kRows &&
                    y[i] - y[i] == 0.f && z[i] - z[i] == 0.f;
    if (!ok) {
      o->valid[i] = 0;
      o->status |= 1;
    }
  }
  return o;
}

void orc_destroy(void* h) { delete (Oracle*)h; }
void orc_set_brute(void* h, int32_t b) { ((Oracle*)h)->brute = b != 0; }
int32_t orc_status(void* h) { return ((Oracle*)h)->status; }
// seconds spent in the FP64 refits of the last run (fit stage, merged refits included)
double orc_fp64_seconds(void* h) { return ((Oracle*)h)->fp64_seconds; }

void orc_run(void* h, int32_t last_stage) {
  Oracle* o = (Oracle*)h;
  o->build_rows();
  if (last_stage >= 1) o->find_neighbours();
  if (last_stage >= 2) o->construct_tracklets();
  if (last_stage >= 3) o->select_tracks();
  if (last_stage >= 4) o->fit_all();
  if (last_stage >= 5) o->merge();
}

// row lists: per slot (job, sector, row) the member indices in ascending index order
int64_t orc_num_slot_members(void* h) { return (int64_t)((Oracle*)h)->slot_idx.size(); }
void orc_get_rows(void* h, int64_t* slot_off, int32_t* members_sorted_by_index) {
  Oracle* o = (Oracle*)h;
  std::copy(o->slot_off.begin(), o->slot_off.end(), slot_off);
  for (size_t s = 0; s + 1 < o->slot_off.size(); ++s) {
    std::vector<int32_t> v(o->slot_idx.begin() + o->slot_off[s], o->slot_idx.begin() + o->slot_off[s + 1]);
    std::sort(v.begin(), v.end());
    std::copy(v.begin(), v.end(), members_sorted_by_index + o->slot_off[s]);
  }
}

void orc_get_links(void* h, int32_t* up_raw, int32_t* down_raw, int32_t* up, int32_t* down) {
  Oracle* o = (Oracle*)h;
  std::copy(o->up_raw.begin(), o->up_raw.end(), up_raw);
  std::copy(o->down_raw.begin(), o->down_raw.end(), down_raw);
  std::copy(o->up.begin(), o->up.end(), up);
  std::copy(o->down.begin(), o->down.end(), down);
}

int32_t orc_num_tracklets(void* h) { return (int32_t)((Oracle*)h)->tracklets.size(); }
int64_t orc_num_tracklet_hits(void* h) {
  int64_t s = 0;
  for (auto& t : ((Oracle*)h)->tracklets) s += t.hits.size();
  return s;
}
// start index, hit CSR (all tracklets, valid or not), state at the last hit
void orc_get_tracklets(void* h, int32_t* start, int32_t* off, int32_t* hits, float* P, float* C,
                       float* x) {
  Oracle* o = (Oracle*)h;
  int64_t k = 0;
  off[0] = 0;
  for (size_t i = 0; i < o->tracklets.size(); ++i) {
    const Tracklet& t = o->tracklets[i];
    start[i] = t.start;
    for (int32_t v : t.hits) hits[k++] = v;
    off[i + 1] = (int32_t)k;
    std::memcpy(P + 5 * i, t.P, sizeof(t.P));
    std::memcpy(C + 15 * i, t.C, sizeof(t.C));
    x[i] = t.x;
  }
}
void orc_get_hitw(void* h, uint64_t* w) {
  Oracle* o = (Oracle*)h;
  std::copy(o->hitw.begin(), o->hitw.end(), w);
}

// tracks after the last stage run; absorbed outer pieces are skipped when merged != 0
int32_t orc_num_tracks(void* h, int32_t merged) {
  int32_t c = 0;
  for (auto& t : ((Oracle*)h)->tracks) c += (!merged || t.merged_into < 0);
  return c;
}
int64_t orc_num_track_hits(void* h, int32_t merged) {
  int64_t c = 0;
  for (auto& t : ((Oracle*)h)->tracks)
    if (!merged || t.merged_into < 0) c += t.hits.size();
  return c;
}
void orc_get_tracks(void* h, int32_t merged, int32_t* tracklet, int32_t* job, int32_t* sector,
                    int32_t* sector2, int32_t* off, int32_t* hits, float* P, float* C, float* x,
                    float* chi2, int32_t* ndf, double* Pd, double* Cd, double* xd, double* chi2d,
                    int32_t* ndfd) {
  Oracle* o = (Oracle*)h;
  int64_t k = 0, m = 0;
  off[0] = 0;
  for (auto& t : o->tracks) {
    if (merged && t.merged_into >= 0) continue;
    tracklet[m] = t.tracklet;
    job[m] = t.job;
    sector[m] = t.sector;
    sector2[m] = t.sector2;
    for (int32_t v : t.hits) hits[k++] = v;
    off[m + 1] = (int32_t)k;
    std::memcpy(P + 5 * m, t.P, sizeof(t.P));
    std::memcpy(C + 15 * m, t.C, sizeof(t.C));
    x[m] = t.x; chi2[m] = t.chi2; ndf[m] = t.ndf;
    std::memcpy(Pd + 5 * m, t.Pd, sizeof(t.Pd));
    std::memcpy(Cd + 15 * m, t.Cd, sizeof(t.Cd));
    xd[m] = t.xd; chi2d[m] = t.chi2d; ndfd[m] = t.ndfd;
    ++m;
  }
}

// A13: hits each output track gained by the downward extension (same order as orc_get_tracks;
// a merged track reports its inner piece's)
void orc_get_track_ext(void* h, int32_t merged, int32_t* n_ext) {
  Oracle* o = (Oracle*)h;
  int64_t m = 0;
  for (auto& t : o->tracks) {
    if (merged && t.merged_into >= 0) continue;
    n_ext[m++] = t.n_ext;
  }
}

// T1: the collision time of every output track (same order as orc_get_tracks), from the
// FP32 fit (t0) and from the FP64 refit (t0d); NaN where the fit failed.
void orc_get_track_t0(void* h, int32_t merged, float* t0, double* t0d) {
  Oracle* o = (Oracle*)h;
  int64_t m = 0;
  for (auto& t : o->tracks) {
    if (merged && t.merged_into >= 0) continue;
    if (!std::isnan(t.t0m)) {  // a chain across the membrane: its link's time (A21)
      t0[m] = t.ndf >= 0 ? t.t0m : NAN;
      t0d[m] = t.ndfd >= 0 ? (double)t.t0m : (double)NAN;
    } else {
      t0[m] = t.ndf >= 0 ? collision_time<float>(o->p, t.P, t.x, t.sector) : NAN;
      t0d[m] = t.ndfd >= 0 ? collision_time<double>(o->p, t.Pd, t.xd, t.sector) : (double)NAN;
    }
    ++m;
  }
}
// T1 alone (pins): the collision time of one state
float orc_collision_time_f32(const float* P, float x, int32_t sector, const Params* p) {
  return collision_time<float>(*p, P, x, sector);
}
double orc_collision_time_f64(const double* P, double x, int32_t sector, const Params* p) {
  return collision_time<double>(*p, P, x, sector);
}

// ---- unit hooks for the pins
// P: 10 values (hi[5], lo[5]) of the compensated state
int32_t orc_propagate_f32(float* P, float* C, float x1, float x2, const Params* p) {
  return propagate<float>(P, P + 5, C, x1, x2, curvature_factor<float>(*p), p->smax);
}
int32_t orc_propagate_f64(double* P, double* C, double x1, double x2, const Params* p) {
  return propagate<double>(P, P + 5, C, x1, x2, curvature_factor<double>(*p), (double)p->smax);
}
int32_t orc_update_f32(float* P, float* C, float my, float mz, const Params* p, float* chi2) {
  return kf_update<float>(P, P + 5, C, my, mz, p->sigma_y * p->sigma_y, p->sigma_z * p->sigma_z, p->smax, chi2);
}
int32_t orc_update_f64(double* P, double* C, double my, double mz, const Params* p, double* chi2) {
  const double sy = p->sigma_y, sz = p->sigma_z;
  return kf_update<double>(P, P + 5, C, my, mz, sy * sy, sz * sz, (double)p->smax, chi2);
}
int32_t orc_rotate_f64(double* P, double* C, double* x, int32_t from, int32_t to, const Params* p) {
  return rotate_sector<double>(P, P + 5, C, *x, from, to, curvature_factor<double>(*p), (double)p->smax);
}
int32_t orc_rotate_f32(float* P, float* C, float* x, int32_t from, int32_t to, const Params* p) {
  return rotate_sector<float>(P, P + 5, C, *x, from, to, curvature_factor<float>(*p), p->smax);
}
void orc_asinc_f32(float u, float* A, float* B) { asinc(u, *A, *B); }
void orc_asinc_f64(double u, double* A, double* B) { asinc(u, *A, *B); }
float orc_row_x(int32_t r) { return kGeo.x[r]; }
float orc_merge_chi2(const float* PA, const float* CA, const float* PB, const float* CB) {
  return Oracle::merge_chi2(PA, CA, PB, CB);
}
// FP64 refit of an arbitrary hit list (inner -> outer, one sector) from given (s, t, k)
int32_t orc_fit_hits_f64(void* h, int32_t nh, const int32_t* hits, const float* stk, double* P,
                         double* C, double* x, double* chi2) {
  Oracle* o = (Oracle*)h;
  std::vector<int32_t> v(hits, hits + nh);
  std::vector<int> hs(nh);
  for (int i = 0; i < nh; ++i) hs[i] = o->sector[hits[i]];
  int32_t ndf;
  return o->fit<double>(v, stk, hs.back(), hs, P, C, *x, *chi2, ndf);
}
int32_t orc_fit_hits_f32(void* h, int32_t nh, const int32_t* hits, const float* stk, float* P,
                         float* C, float* x, float* chi2) {
  Oracle* o = (Oracle*)h;
  std::vector<int32_t> v(hits, hits + nh);
  std::vector<int> hs(nh);
  for (int i = 0; i < nh; ++i) hs[i] = o->sector[hits[i]];
  int32_t ndf;
  return o->fit<float>(v, stk, hs.back(), hs, P, C, *x, *chi2, ndf);
}

// ---------------------------------------------------------------- A25: looper leg pairs
// A looper's two legs are tracked separately, each along increasing x (the return leg against
// its momentum), so they describe the same circle with opposite signed curvature and opposite
// tan(lambda), and both run towards the circle's point farthest from the beam line, where the
// looper turned.  Reading: among fitted output tracks of one event and one z side whose
// circles turn inside the chamber (2R < 245 cm / cos 10 deg), A and B pair when their
// curvatures and tan(lambda) have opposite signs, their circle centres (global x, y) agree
// within LEG_GATE in each coordinate, and so do their z extrapolated along the helix to that
// turning point; the score is the sum of the three squared differences, pairs are mutual
// best ones (ties: smaller output index).  Which leg left the vertex is not decided.
// Geometry in FP32, in this order: C = cb k; c = sqrt((1 - s)(1 + s)); local centre
// (x - s/C, y + c/C); global by the sector angle (x ca - y sa, x sa + y ca); R = 1/|C|; the
// turning point centre + R centre/|centre|; the chord from the track's point to it; the arc
// chord A(u), u = min(1, chord |C| / 2) with the FP32 asin(u)/u of R5; z + t arc.
constexpr float kLegGate = 3.0f;
struct LegGeo {
  bool looper;
  float cx, cy, zt, C, t;
};
LegGeo leg_geometry(const Params& p, const float* P, float x, int sector) {
  LegGeo L{};
  const float C = curvature_factor<float>(p) * P[4];
  const float cmin = (float)(2.0 / (245.0 / std::cos(10.0 * 3.14159265358979323846 / 180.0)));
  L.looper = std::fabs(C) > cmin;
  if (!L.looper) return L;
  const double al = (10.0 + 20.0 * (double)(sector % kRowsPerSide)) * 3.14159265358979323846 / 180.0;
  const float ca = (float)std::cos(al), sa = (float)std::sin(al);
  const float s = P[2];
  const float c = std::sqrt((1.0f - s) * (1.0f + s));
  const float lx = x - s / C, ly = P[0] + c / C;
  L.cx = lx * ca - ly * sa;
  L.cy = lx * sa + ly * ca;
  if (!std::isfinite(L.cx) || !std::isfinite(L.cy)) {  // no circle: not a looper
    L.looper = false;
    return L;
  }
  const float R = 1.0f / std::fabs(C);
  const float cn = std::sqrt(L.cx * L.cx + L.cy * L.cy);
  const float tx = L.cx + R * (L.cx / cn), ty = L.cy + R * (L.cy / cn);
  const float px = x * ca - P[0] * sa, py = x * sa + P[0] * ca;
  const float dx = tx - px, dy = ty - py;
  const float chord = std::sqrt(dx * dx + dy * dy);
  const float u = std::fmin(1.0f, chord * std::fabs(C) * 0.5f);
  float A, B;
  asinc(u, A, B);
  L.zt = P[1] + P[3] * (chord * A);
  L.C = C;
  L.t = P[3];
  return L;
}

// leg[i] = the output index of track i's other leg, or -1.  brute: every pair of tracks is
// compared instead of the tracks of the 3 x 3 centre cells (the same pairs result).
void orc_pair_legs(const Params* p, int32_t K, const float* param, const float* x_ref, const int32_t* sector,
                   const int32_t* event, const int32_t* ndf, int32_t* leg, int32_t brute) {
  std::vector<LegGeo> G(K);
  for (int i = 0; i < K; ++i) {
    G[i] = LegGeo{};
    if (ndf[i] >= 0) G[i] = leg_geometry(*p, param + 5 * i, x_ref[i], sector[i]);
  }
  // candidates by (event, side, 4-cm cell of the centre)
  std::unordered_map<int64_t, std::vector<int32_t>> cells;
  auto key = [&](int i, int dx, int dy) {
    const int64_t ix = (int64_t)std::floor(G[i].cx / 4.0f) + dx, iy = (int64_t)std::floor(G[i].cy / 4.0f) + dy;
    return (((int64_t)event[i] * 2 + (sector[i] >= kRowsPerSide)) * 4096 + (ix & 4095)) * 4096 + (iy & 4095);
  };
  for (int i = 0; i < K; ++i)
    if (G[i].looper) cells[key(i, 0, 0)].push_back(i);
  std::vector<float> best(K, 0.f);
  std::vector<int32_t> arg(K, -1);
  std::vector<int32_t> all;
  if (brute)
    for (int i = 0; i < K; ++i)
      if (G[i].looper) all.push_back(i);
  for (int a = 0; a < K; ++a) {
    if (!G[a].looper) continue;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        const std::vector<int32_t>* list = &all;
        if (!brute) {
          const auto it = cells.find(key(a, dx, dy));
          if (it == cells.end()) continue;
          list = &it->second;
        } else if (dx != 0 || dy != 0) {
          continue;
        }
        for (const int b : *list) {
          if (b == a || event[b] != event[a] || (sector[b] >= kRowsPerSide) != (sector[a] >= kRowsPerSide)) continue;
          if (!(G[a].C * G[b].C < 0.f) || !(G[a].t * G[b].t <= 0.f)) continue;
          const float ex = G[a].cx - G[b].cx, ey = G[a].cy - G[b].cy, ez = G[a].zt - G[b].zt;
          if (!(std::fabs(ex) <= kLegGate) || !(std::fabs(ey) <= kLegGate) || !(std::fabs(ez) <= kLegGate)) continue;
          const float sc = (ex * ex + ey * ey) + ez * ez;
          if (arg[a] < 0 || sc < best[a] || (sc == best[a] && b < arg[a])) { best[a] = sc; arg[a] = b; }
        }
      }
  }
  for (int i = 0; i < K; ++i) leg[i] = (arg[i] >= 0 && arg[arg[i]] == i) ? arg[i] : -1;
}

// C2-C4: encode n clusters against K tracks.  Writes H + U records (H = off[K] track
// hits, U = clusters in no track); returns that count; *status gets 1 for C3's cases.
int32_t orc_compress(const Params* p, int32_t n, const uint8_t* sector, const int16_t* row,
                     const float* y, const float* z, int32_t K, const int32_t* off, const int32_t* hits,
                     const float* param, const float* x_ref, const int32_t* tsec, const int32_t* ndf,
                     float q_y, float q_z, uint16_t* rs, int16_t* ey, int16_t* ez, int8_t* ezh,
                     int32_t* status) {
  const float iy = 1.0f / q_y, iz = 1.0f / q_z;
  int32_t st = 0;
  std::vector<uint8_t> in_track(n, 0);
  int32_t m = 0;
  auto put_abs = [&](int32_t h) {
    if (ezh) ezh[m] = 0;
    if (!cluster_ok(sector[h], row[h], y[h], z[h])) {
      rs[m] = kRecInvalid; ey[m] = 0; ez[m] = 0; st |= 1;
      return;
    }
    rs[m] = (uint16_t)(row[h] | (sector[h] << 8) | (1 << 15));
    ey[m] = abs_code(y[h], iy, st);
    if (ezh)
      abs_code_wide(z[h], iz, ez[m], ezh[m], st);
    else
      ez[m] = abs_code(z[h], iz, st);
  };
  for (int32_t i = 0; i < K; ++i) {
    for (int32_t j = off[i]; j < off[i + 1]; ++j, ++m) {
      const int32_t h = hits[j];
      if (ezh) ezh[m] = 0;
      if (h < 0 || h >= n) { rs[m] = kRecInvalid; ey[m] = 0; ez[m] = 0; st |= 1; continue; }
      in_track[h] = 1;
      if (!cluster_ok(sector[h], row[h], y[h], z[h])) { put_abs(h); continue; }
      float py, pz;
      if (ndf[i] >= 0 && predict(*p, param + 5 * i, x_ref[i], tsec[i], sector[h], row[h], py, pz)) {
        const float e1 = std::rint((y[h] - py) * iy);
        const float e2 = std::rint((z[h] - pz) * iz);
        if (std::fabs(e1) <= (float)kCodeMax && std::fabs(e2) <= (float)kCodeMax) {
          rs[m] = (uint16_t)(row[h] | (sector[h] << 8));
          ey[m] = (int16_t)e1;
          ez[m] = (int16_t)e2;
          continue;
        }
      }
      put_abs(h);
    }
  }
  for (int32_t h = 0; h < n; ++h)
    if (!in_track[h]) { put_abs(h); ++m; }
  *status = st;
  return m;
}

// C5: decode m records; the first off[K] belong to the tracks in order.
void orc_decompress(const Params* p, int32_t K, const int32_t* off, const float* param,
                    const float* x_ref, const int32_t* tsec, const int32_t* ndf, int32_t m,
                    const uint16_t* rs, const int16_t* ey, const int16_t* ez, const int8_t* ezh,
                    float q_y, float q_z, uint8_t* sector, int16_t* row, float* y, float* z) {
  int32_t i = 0;
  for (int32_t j = 0; j < m; ++j) {
    while (i < K && j >= off[i + 1]) ++i;
    const int r = rs[j] & 0xFF, s = (rs[j] >> 8) & 0x7F;
    const bool absolute = (rs[j] >> 15) != 0;
    if (r >= kRows || s >= kSectors) {
      sector[j] = 255; row[j] = -1; y[j] = NAN; z[j] = NAN;
      continue;
    }
    sector[j] = (uint8_t)s;
    row[j] = (int16_t)r;
    const int32_t cz = (absolute && ezh) ? (int32_t)ezh[j] * 65536 + (int32_t)(uint16_t)ez[j] : (int32_t)ez[j];
    const float dy = (float)ey[j] * q_y, dz = (float)cz * q_z;
    float py = 0.f, pz = 0.f;
    if (!absolute) {
      if (!(i < K && ndf[i] >= 0 && predict(*p, param + 5 * i, x_ref[i], tsec[i], s, r, py, pz))) {
        y[j] = NAN; z[j] = NAN;
        continue;
      }
      y[j] = py + dy;
      z[j] = pz + dz;
    } else {
      y[j] = dy;
      z[j] = dz;
    }
  }
}

// E1: the normalised frequencies freq[65536] of a stream of n symbols.
void orc_rans_model(const uint16_t* sym, int32_t n, uint32_t* freq) {
  std::vector<int64_t> c(kRansM, 0);
  for (int32_t i = 0; i < n; ++i) ++c[sym[i]];
  int64_t K = 0;
  uint32_t top = 0;
  for (uint32_t v = 0; v < kRansM; ++v) {
    if (c[v] > 0) ++K;
    if (c[v] > c[top]) top = v;
  }
  uint64_t sum = 0;
  for (uint32_t v = 0; v < kRansM; ++v) {
    freq[v] = c[v] > 0 ? (uint32_t)std::max<int64_t>(1, c[v] * ((int64_t)kRansM - K) / n) : 0;
    sum += freq[v];
  }
  if (n > 0) freq[top] += (uint32_t)(kRansM - sum);
}

// E2, E4, E5: encodes with the given model; returns the number of words and fills
// lane_off[lanes + 1] and words[] (capacity: lanes * (S + 2)).
int32_t orc_rans_encode(const uint16_t* sym, int32_t n, const uint32_t* freq, uint32_t* lane_off,
                        uint16_t* words) {
  std::vector<uint32_t> C(kRansM + 1, 0);
  for (uint32_t v = 0; v < kRansM; ++v) C[v + 1] = C[v] + freq[v];
  const int64_t lanes = rans_lanes(n);
  int64_t pos = 0;
  std::vector<uint16_t> out;
  for (int64_t l = 0; l < lanes; ++l) {
    lane_off[l] = (uint32_t)pos;
    int64_t first, count;
    rans_lane(n, l, first, count);
    if (count == 0) continue;
    uint32_t x = kRansL;
    out.clear();
    for (int64_t m = count - 1; m >= 0; --m) {
      const uint16_t s = sym[first + kRansLanesPerChunk * m];
      const uint32_t f = freq[s];
      if ((uint64_t)x >= (uint64_t)f << 16) {
        out.push_back((uint16_t)(x & 0xFFFF));
        x >>= 16;
      }
      x = ((x / f) << 16) + (x % f) + C[s];
    }
    words[pos++] = (uint16_t)(x >> 16);
    words[pos++] = (uint16_t)(x & 0xFFFF);
    for (auto it = out.rbegin(); it != out.rend(); ++it) words[pos++] = *it;
  }
  lane_off[lanes] = (uint32_t)pos;
  return (int32_t)pos;
}

// E3: decodes n symbols.
void orc_rans_decode(const uint32_t* freq, const uint32_t* lane_off, const uint16_t* words, int32_t n,
                     uint16_t* sym) {
  std::vector<uint32_t> C(kRansM + 1, 0);
  for (uint32_t v = 0; v < kRansM; ++v) C[v + 1] = C[v] + freq[v];
  const int64_t lanes = rans_lanes(n);
  for (int64_t l = 0; l < lanes; ++l) {
    int64_t first, count;
    rans_lane(n, l, first, count);
    if (count == 0) continue;
    int64_t p = lane_off[l];
    uint32_t x = ((uint32_t)words[p] << 16) | words[p + 1];
    p += 2;
    for (int64_t m = 0; m < count; ++m) {
      const uint32_t slot = x & 0xFFFF;
      // the symbol whose interval [C_s, C_s + f_s) holds the slot
      const uint32_t s = (uint32_t)(std::upper_bound(C.begin(), C.end() - 1, slot) - C.begin()) - 1;
      sym[first + kRansLanesPerChunk * m] = (uint16_t)s;
      x = freq[s] * (x >> 16) + slot - C[s];
      if (x < kRansL) x = (x << 16) | words[p++];
    }
  }
}

int64_t orc_rans_lanes(int64_t n) { return rans_lanes(n); }

// F1-F6: the clusters of n digits; returns their number (<= n).
int32_t orc_find_clusters(int32_t n, const uint8_t* sector, const int16_t* row, const int16_t* pad,
                          const int16_t* time, const uint16_t* adc, float pitch, float bin, int32_t n_time,
                          int32_t q_min, int32_t* digit, uint8_t* csec, int16_t* crow, float* y, float* z,
                          uint32_t* qtot, uint32_t* qmax, float* spad, float* stime, int32_t* status) {
  int32_t P[kRows];
  for (int r = 0; r < kRows; ++r) P[r] = cf_pads(r, pitch);
  auto in_range = [&](int s, int r, int p, int t) {
    return s >= 0 && s < kSectors && r >= 0 && r < kRows && p >= 0 && p < P[r] && t >= 0 && t < n_time;
  };
  auto key = [&](int s, int r, int p, int t) {
    return (((uint64_t)s * kRows + (uint64_t)r) * 1024 + (uint64_t)p) * 65536 + (uint64_t)t;
  };
  std::unordered_map<uint64_t, uint32_t> map;
  int32_t st = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!in_range(sector[i], row[i], pad[i], time[i])) { st |= 1; continue; }
    map[key(sector[i], row[i], pad[i], time[i])] += adc[i];
  }
  auto charge = [&](int s, int r, int p, int t) -> uint32_t {
    if (!in_range(s, r, p, t)) return 0;
    auto it = map.find(key(s, r, p, t));
    return it == map.end() ? 0 : it->second;
  };
  int32_t m = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int s = sector[i], r = row[i], p = pad[i], t = time[i];
    if (!in_range(s, r, p, t)) continue;
    const uint32_t q = charge(s, r, p, t);
    if (q < (uint32_t)q_min) continue;
    bool peak = true;
    for (int dp = -1; dp <= 1 && peak; ++dp)
      for (int dt = -1; dt <= 1 && peak; ++dt) {
        if (dp == 0 && dt == 0) continue;
        const uint32_t qn = charge(s, r, p + dp, t + dt);
        const bool before = dp < 0 || (dp == 0 && dt < 0);
        if (before ? !(q > qn) : !(q >= qn)) peak = false;
      }
    if (!peak) continue;
    int64_t Q = 0, Sp = 0, St = 0, Spp = 0, Stt = 0;
    for (int dp = -1; dp <= 1; ++dp)
      for (int dt = -1; dt <= 1; ++dt) {
        const int64_t qn = charge(s, r, p + dp, t + dt);
        Q += qn;
        Sp += qn * dp;
        St += qn * dt;
        Spp += qn * dp * dp;
        Stt += qn * dt * dt;
      }
    const float fq = (float)Q;
    const float mp = (float)Sp / fq, mt = (float)St / fq;
    const float vp = (float)Spp / fq - mp * mp, vt = (float)Stt / fq - mt * mt;
    const float half = (float)((double)P[r] * (double)pitch / 2.0);
    digit[m] = i;
    csec[m] = (uint8_t)s;
    crow[m] = (int16_t)r;
    y[m] = ((float)p + mp + 0.5f) * pitch - half;
    const float az = ((float)t + mt + 0.5f) * bin;
    z[m] = s < kRowsPerSide ? az : -az;
    qtot[m] = (uint32_t)Q;
    qmax[m] = q;
    spad[m] = std::sqrt(vp > 0.f ? vp : 0.f);
    stime[m] = std::sqrt(vt > 0.f ? vt : 0.f);
    ++m;
  }
  *status = st;
  return m;
}

int32_t orc_cf_pads(int32_t r, float pitch) { return cf_pads(r, pitch); }

// C1 alone (pins): returns 1 and (py, pz) when there is a prediction.
int32_t orc_predict(const Params* p, const float* P, float xref, int32_t sref, int32_t sec, int32_t row,
                    float* pyz) {
  return predict(*p, P, xref, sref, sec, row, pyz[0], pyz[1]);
}

}  // extern "C"
