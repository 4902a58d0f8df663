// Serial coordinate-descent FCI oracle -- TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark load this library.  It shares no code with the HIP path.
//
// What it computes (paper: Sec. 3.1, Algorithm 1 "CDFCI"; Sec. 4.1.1 get_column /
// get_entry; Appendix A for the line search):
//   * determinants are (a, b) occupation strings; spin-orbital order is all
//     alpha orbitals then all beta orbitals, |a,b> = prod_{P asc} a+_P |0>;
//   * Slater-Condon entries of eq. (entry): the phase of the excitation
//     operator (a+_r a_p, or a+_r a+_s a_q a_p) is found by applying it to the
//     ket one operator at a time, the value from h and the chemist integrals
//     with v_PQRS = (PR|QS) for matching spins;
//   * Algorithm 1 in its order: select i = argmax over the candidate set of
//     |4 b_i + 4 mu c_i| (ties: smaller (b, a) as an unsigned 128-bit number),
//     exact line search of the quartic, c_i += eta, b += eta H_{:,i} with the
//     compression rule (update b_j only if c_j != 0 or |eta H_ji| >= tau),
//     recalculation b_i = sum_j H_ji c_j, then mu and alpha from the pre-step
//     c_i, b_i (kept in __float128 as the paper keeps them in quad precision),
//     energy alpha/mu and the damped step accumulator d.
//   * candidates of the next step are the column of the chosen coordinate
//     (entries with H_ji != 0) plus the coordinate itself.
//   * b^(0) = H c^(0) exactly (no compression in the initialisation).

#include <quadmath.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace {

struct Key {
  uint64_t a, b;
  bool operator==(const Key& o) const { return a == o.a && b == o.b; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    return std::hash<uint64_t>()(k.a) * 1000003u ^ std::hash<uint64_t>()(k.b);
  }
};
// ordering for ties: (b, a) as an unsigned 128-bit value
bool key_less(const Key& x, const Key& y) { return x.b != y.b ? x.b < y.b : x.a < y.a; }

struct Ham {
  int N;
  const double* h;
  const double* eri;
  double one(int P, int Q) const {  // spin-orbital one-body integral
    if ((P >= N) != (Q >= N)) return 0.0;
    return h[(P % N) * N + (Q % N)];
  }
  double chem(int p, int q, int r, int s) const {  // spatial (pq|rs)
    return eri[((size_t)(p * N + q) * N + r) * N + s];
  }
  double v(int P, int Q, int R, int S) const {  // <PQ|RS> = (PR|QS)
    if ((P >= N) != (R >= N) || (Q >= N) != (S >= N)) return 0.0;
    return chem(P % N, R % N, Q % N, S % N);
  }
};

// spin-orbital occupation of a determinant
struct Occ {
  uint64_t w[2];  // w[0]: alpha (spin-orbitals 0..N-1), w[1]: beta (N..2N-1)
};
inline bool is_set(const Occ& x, int P, int N) {
  return P < N ? (x.w[0] >> P) & 1 : (x.w[1] >> (P - N)) & 1;
}
inline int count_below(const Occ& x, int P, int N) {
  if (P < N) return __builtin_popcountll(x.w[0] & ((P ? (~0ull >> (64 - P)) : 0ull)));
  int Q = P - N;
  return __builtin_popcountll(x.w[0]) + __builtin_popcountll(x.w[1] & (Q ? (~0ull >> (64 - Q)) : 0ull));
}
inline void flip(Occ& x, int P, int N) {
  if (P < N)
    x.w[0] ^= 1ull << P;
  else
    x.w[1] ^= 1ull << (P - N);
}
// apply an operator string right-to-left; kinds: 'c' create, 'a' annihilate
int apply_ops(Occ& x, int n, const char* kind, const int* idx, int N) {
  int sign = 1;
  for (int t = n - 1; t >= 0; --t) {
    int P = idx[t];
    bool o = is_set(x, P, N);
    if ((kind[t] == 'a') != o) return 0;
    if (count_below(x, P, N) & 1) sign = -sign;
    flip(x, P, N);
  }
  return sign;
}

std::vector<int> occ_list(const Occ& x, int N) {
  std::vector<int> out;
  for (int P = 0; P < 2 * N; ++P)
    if (is_set(x, P, N)) out.push_back(P);
  return out;
}

double diag_entry(const Ham& H, const Occ& x) {
  std::vector<int> oc = occ_list(x, H.N);
  double e = 0.0;
  for (int P : oc) e += H.one(P, P);
  double two = 0.0;
  for (int P : oc)
    for (int Q : oc) two += H.v(P, Q, P, Q) - H.v(P, Q, Q, P);
  return e + 0.5 * two;
}

struct Elem {
  Key k;
  double v;
};

// get_column: diagonal first, then all singles and doubles (zeros kept)
void column(const Ham& H, Key key, std::vector<Elem>& out) {
  const int N = H.N;
  out.clear();
  Occ x{{key.a, key.b}};
  out.push_back({key, diag_entry(H, x)});
  std::vector<int> oc = occ_list(x, N), vi;
  for (int P = 0; P < 2 * N; ++P)
    if (!is_set(x, P, N)) vi.push_back(P);
  for (int p : oc)
    for (int r : vi) {
      if ((p >= N) != (r >= N)) continue;
      Occ y = x;
      const char kd[2] = {'c', 'a'};
      const int ix[2] = {r, p};
      int s = apply_ops(y, 2, kd, ix, N);
      double val = H.one(r, p);
      for (int k : oc) val += H.v(r, k, p, k) - H.v(r, k, k, p);
      out.push_back({Key{y.w[0], y.w[1]}, s * val});
    }
  for (size_t i = 0; i < oc.size(); ++i)
    for (size_t j = i + 1; j < oc.size(); ++j)
      for (size_t u = 0; u < vi.size(); ++u)
        for (size_t w = u + 1; w < vi.size(); ++w) {
          int p = oc[i], q = oc[j], r = vi[u], s = vi[w];
          int sp = (p >= N) + (q >= N), sr = (r >= N) + (s >= N);
          if (sp != sr) continue;
          // for a mixed-spin pair, p < q and r < s put the alpha index first
          // in both, so spin is conserved per electron
          Occ y = x;
          const char kd[4] = {'c', 'c', 'a', 'a'};
          const int ix[4] = {r, s, q, p};
          int sg = apply_ops(y, 4, kd, ix, N);
          double val = H.v(r, s, p, q) - H.v(r, s, q, p);
          out.push_back({Key{y.w[0], y.w[1]}, sg * val});
        }
}

// ---- exact line search (Appendix A): argmin over the real critical points
long double hq(long double e, long double v1, long double v2, long double v3) {
  return ((e + v3) * e + v2) * e * e + v1 * e;
}
double line_search(double v1d, double v2d, double v3d) {
  long double v1 = v1d, v2 = v2d, v3 = v3d;
  // cubic 4 e^3 + 3 v3 e^2 + 2 v2 e + v1 = 0, normalised: e^3 + B e^2 + C e + D
  long double B = 0.75L * v3, C = 0.5L * v2, D = 0.25L * v1;
  long double p = C - B * B / 3.0L;
  long double q = 2.0L * B * B * B / 27.0L - B * C / 3.0L + D;
  long double disc = (q / 2) * (q / 2) + (p / 3) * (p / 3) * (p / 3);
  std::vector<long double> roots;
  if (disc > 0) {
    long double sd = sqrtl(disc);
    roots.push_back(cbrtl(-q / 2 + sd) + cbrtl(-q / 2 - sd) - B / 3);
  } else if (p == 0) {
    roots.push_back(-B / 3);
  } else {
    long double m = 2.0L * sqrtl(-p / 3.0L);
    long double arg = (3.0L * q / (2.0L * p)) * sqrtl(-3.0L / p);
    if (arg > 1) arg = 1;
    if (arg < -1) arg = -1;
    long double th = acosl(arg) / 3.0L;
    for (int k = 0; k < 3; ++k) roots.push_back(m * cosl(th - 2.0L * (long double)M_PI * k / 3.0L) - B / 3);
  }
  long double best = 0, bh = 0;
  bool have = false;
  for (long double r : roots) {
    for (int it = 0; it < 16; ++it) {  // Newton polish on the cubic
      long double f = ((4 * r + 3 * v3) * r + 2 * v2) * r + v1;
      long double fp = (12 * r + 6 * v3) * r + 2 * v2;
      if (fp == 0) break;
      long double dr = f / fp;
      r -= dr;
      if (fabsl(dr) <= 1e-19L * fabsl(r)) break;
    }
    long double hv = hq(r, v1, v2, v3);
    if (!have || hv < bh || (hv == bh && fabsl(r) < fabsl(best))) {
      best = r;
      bh = hv;
      have = true;
    }
  }
  return (double)best;
}

struct Val {
  double c = 0.0, b = 0.0;
};

}  // namespace

extern "C" {

// Spin-summed reduced density matrices of the normalised vector c over the
// given determinants (RDMs of Sec. 3.4, eq. (subopt)):
//   g1[p*N+q]           = sum_s <a+_ps a_qs>
//   g2[((p*N+q)*N+r)*N+s] = sum_st <a+_ps a+_rt a_st a_qs>
// by applying every operator string to every determinant of the support and
// looking the result up (annihilators must hit occupied spin-orbitals, so Q and
// S range over the occupied ones and P, R over the empty ones plus Q, S).
int oracle_rdm12(int N, int64_t ndet, const uint64_t* ka, const uint64_t* kb, const double* c,
                 double* g1, double* g2) {
  if (N < 1 || N > 64 || ndet < 1) return -1;
  std::unordered_map<Key, double, KeyHash> sup;
  double nrm = 0.0;
  for (int64_t i = 0; i < ndet; ++i) nrm += c[i] * c[i];
  nrm = sqrt(nrm);
  for (int64_t i = 0; i < ndet; ++i) sup[Key{ka[i], kb[i]}] += c[i] / nrm;
  const size_t N2 = (size_t)N * N, N4 = N2 * N2;
  for (size_t i = 0; i < N2; ++i) g1[i] = 0.0;
  for (size_t i = 0; i < N4; ++i) g2[i] = 0.0;
  const int ns = 2 * N;
  for (const auto& kv : sup) {
    const Occ x{{kv.first.a, kv.first.b}};
    const double cj = kv.second;
    std::vector<int> oc = occ_list(x, N);
    for (int Q : oc)
      for (int P = 0; P < ns; ++P) {
        if ((P >= N) != (Q >= N)) continue;
        if (P != Q && is_set(x, P, N)) continue;
        Occ y = x;
        const char kd[2] = {'c', 'a'};
        const int ix[2] = {P, Q};
        int sg = apply_ops(y, 2, kd, ix, N);
        if (!sg) continue;
        auto it = sup.find(Key{y.w[0], y.w[1]});
        if (it == sup.end()) continue;
        g1[(P % N) * N + (Q % N)] += it->second * sg * cj;
      }
    for (int Q : oc)
      for (int S : oc) {
        if (Q == S) continue;
        for (int P = 0; P < ns; ++P) {
          if ((P >= N) != (Q >= N)) continue;
          if (P != Q && P != S && is_set(x, P, N)) continue;
          for (int R = 0; R < ns; ++R) {
            if ((R >= N) != (S >= N)) continue;
            if (R == P) continue;
            if (R != Q && R != S && is_set(x, R, N)) continue;
            Occ y = x;
            const char kd[4] = {'c', 'c', 'a', 'a'};
            const int ix[4] = {P, R, S, Q};
            int sg = apply_ops(y, 4, kd, ix, N);
            if (!sg) continue;
            auto it = sup.find(Key{y.w[0], y.w[1]});
            if (it == sup.end()) continue;
            g2[(((size_t)(P % N) * N + (Q % N)) * N + (R % N)) * N + (S % N)] += it->second * sg * cj;
          }
        }
      }
  }
  return 0;
}

// c^T H c / c^T c over the given support (integrals may be perturbed by the
// caller): each support column from get_column, entries looked up in the support
double oracle_support_energy(int N, const double* h, const double* eri, int64_t ndet,
                             const uint64_t* ka, const uint64_t* kb, const double* c) {
  Ham H{N, h, eri};
  std::unordered_map<Key, double, KeyHash> sup;
  for (int64_t i = 0; i < ndet; ++i) sup[Key{ka[i], kb[i]}] += c[i];
  std::vector<Elem> col;
  long double num = 0.0L, den = 0.0L;
  for (const auto& kv : sup) {
    column(H, kv.first, col);
    for (const Elem& e : col) {
      auto it = sup.find(e.k);
      if (it != sup.end()) num += (long double)it->second * e.v * kv.second;
    }
    den += (long double)kv.second * kv.second;
  }
  return (double)(num / den);
}

double oracle_line_search(double v1, double v2, double v3) { return line_search(v1, v2, v3); }

double oracle_entry(int N, const double* h, const double* eri, uint64_t bra_a, uint64_t bra_b,
                    uint64_t ket_a, uint64_t ket_b) {
  Ham H{N, h, eri};
  std::vector<Elem> col;
  column(H, Key{ket_a, ket_b}, col);
  for (const Elem& e : col)
    if (e.k.a == bra_a && e.k.b == bra_b) return e.v;
  return 0.0;
}

// get_column into caller arrays; returns the number of entries (diagonal first)
// or -needed if cap is too small
int64_t oracle_column(int N, const double* h, const double* eri, uint64_t a, uint64_t b, int64_t cap,
                      uint64_t* out_a, uint64_t* out_b, double* out_v) {
  Ham H{N, h, eri};
  std::vector<Elem> col;
  column(H, Key{a, b}, col);
  if ((int64_t)col.size() > cap) return -(int64_t)col.size();
  for (size_t i = 0; i < col.size(); ++i) {
    out_a[i] = col[i].k.a;
    out_b[i] = col[i].k.b;
    out_v[i] = col[i].v;
  }
  return (int64_t)col.size();
}

// Algorithm 1.  Returns 0 on success, -1 on bad input, -2 if the trajectory
// hits mu <= 0.  Optional per-step outputs (length max_steps) may be NULL.
int oracle_cd_run(int N, const double* h, const double* eri, int ninit, const uint64_t* init_a,
                  const uint64_t* init_b, const double* init_c, double tau, int64_t max_steps,
                  double theta, double dx_tol, double* traj_E, uint64_t* traj_a, uint64_t* traj_b,
                  double* traj_eta, double* traj_gap, int64_t* steps_done, double* mu_out,
                  double* alpha_out, int64_t* nstored, int64_t* elements, int64_t cap,
                  uint64_t* out_a, uint64_t* out_b, double* out_c, double* out_bv) {
  if (N < 1 || N > 64 || ninit < 1) return -1;
  Ham H{N, h, eri};
  std::unordered_map<Key, Val, KeyHash> wf;
  wf.reserve(1 << 16);
  std::vector<Elem> col;
  std::vector<Key> cand;
  int64_t nelem = 0;

  // initial state: c^(0) given, b^(0) = H c^(0) exactly
  for (int t = 0; t < ninit; ++t) wf[Key{init_a[t], init_b[t]}].c += init_c[t];
  for (int t = 0; t < ninit; ++t) {
    Key D{init_a[t], init_b[t]};
    column(H, D, col);
    for (const Elem& e : col) {
      if (e.v == 0.0) continue;
      wf[e.k].b += init_c[t] * e.v;
      cand.push_back(e.k);
    }
  }
  std::sort(cand.begin(), cand.end(), key_less);
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  __float128 mu = 0, alpha = 0;
  for (auto& kv : wf) {
    mu += (__float128)kv.second.c * kv.second.c;
    alpha += (__float128)kv.second.c * kv.second.b;
  }
  double d = 0.0;
  int64_t step = 0;
  for (; step < max_steps; ++step) {
    // select: largest |g| with ties to the smaller (b, a); also track the runner-up
    double mud = (double)mu;
    Key best{0, 0}, second{0, 0};
    double gbest = -1.0, g2 = -1.0;
    for (const Key& k : cand) {
      auto it = wf.find(k);
      double c = it == wf.end() ? 0.0 : it->second.c;
      double b = it == wf.end() ? 0.0 : it->second.b;
      double g = fabs(4.0 * b + 4.0 * mud * c);
      if (g > gbest || (g == gbest && key_less(k, best))) {
        second = best;
        g2 = gbest;
        best = k;
        gbest = g;
      } else if (g > g2 || (g == g2 && key_less(k, second))) {
        second = k;
        g2 = g;
      }
    }
    Key I = best;
    Val& vi = wf[I];
    double ci = vi.c, bi = vi.b;
    double Hii = diag_entry(H, Occ{{I.a, I.b}});
    double eta = line_search(4.0 * bi + 4.0 * mud * ci, 2.0 * Hii + 4.0 * ci * ci + 2.0 * mud, 4.0 * ci);
    // update c and b (compression rule), then recalculate b_i
    vi.c = ci + eta;
    column(H, I, col);
    nelem += (int64_t)col.size();
    cand.clear();
    double recalc = 0.0;
    for (size_t t = 0; t < col.size(); ++t) {
      const Elem& e = col[t];
      if (t == 0) {
        recalc += e.v * (ci + eta);
        cand.push_back(I);
        continue;
      }
      if (e.v == 0.0) continue;
      cand.push_back(e.k);
      double delta = eta * e.v;
      auto it = wf.find(e.k);
      double cj = it == wf.end() ? 0.0 : it->second.c;
      if (cj != 0.0 || fabs(delta) >= tau) {
        if (it == wf.end()) it = wf.emplace(e.k, Val{}).first;
        it->second.b += delta;
      }
      recalc += e.v * cj;
    }
    Val& vi2 = wf[I];
    vi2.b = recalc;
    mu += 2 * (__float128)eta * ci + (__float128)eta * eta;
    alpha += 2 * (__float128)eta * bi + (__float128)eta * eta * Hii;
    if (mu <= 0) return -2;
    // damped accumulator, seeded by the first step
    d = step == 0 ? fabs(eta) : theta * d + (1.0 - theta) * fabs(eta);
    if (traj_E) traj_E[step] = (double)(alpha / mu);
    if (traj_a) traj_a[step] = I.a;
    if (traj_b) traj_b[step] = I.b;
    if (traj_eta) traj_eta[step] = eta;
    if (traj_gap) traj_gap[step] = gbest > 0 ? (gbest - (g2 < 0 ? 0 : g2)) / gbest : 0.0;
    if (d < dx_tol) {
      ++step;
      break;
    }
  }
  *steps_done = step;
  *mu_out = (double)mu;
  *alpha_out = (double)alpha;
  *nstored = (int64_t)wf.size();
  *elements = nelem;
  if (cap > 0) {
    int64_t t = 0;
    for (auto& kv : wf) {
      if (t >= cap) break;
      out_a[t] = kv.first.a;
      out_b[t] = kv.first.b;
      out_c[t] = kv.second.c;
      out_bv[t] = kv.second.b;
      ++t;
    }
  }
  return 0;
}

// The same Algorithm 1 on several host threads (OpenMP), for the CPU timing
// baseline: the column of the chosen coordinate is generated in independent
// pieces (one per occupied orbital for singles, one per occupied pair for
// doubles) and joined in the serial order, the lookups and the b updates of
// the column's entries run in parallel (the entries of one column are
// distinct determinants, so each stored value has one writer; new entries are
// inserted afterwards in column order), the recalculation sum and the
// selection are reduced in the serial order.  Every value, and so the whole
// trajectory, is bit for bit that of oracle_cd_run.
static void column_mt(const Ham& H, Key key, std::vector<Elem>& out, int threads) {
  const int N = H.N;
  Occ x{{key.a, key.b}};
  std::vector<int> oc = occ_list(x, N), vi;
  for (int P = 0; P < 2 * N; ++P)
    if (!is_set(x, P, N)) vi.push_back(P);
  const int no = (int)oc.size();
  std::vector<std::pair<int, int>> pairs;
  for (int i = 0; i < no; ++i)
    for (int j = i + 1; j < no; ++j) pairs.push_back({i, j});
  // piece 0..no-1: singles of oc[i]; piece no + t: doubles of pair t
  const int npieces = no + (int)pairs.size();
  std::vector<std::vector<Elem>> piece(npieces);
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
  for (int t = 0; t < npieces; ++t) {
    std::vector<Elem>& o = piece[t];
    if (t < no) {
      const int p = oc[t];
      for (int r : vi) {
        if ((p >= N) != (r >= N)) continue;
        Occ y = x;
        const char kd[2] = {'c', 'a'};
        const int ix[2] = {r, p};
        int sg = apply_ops(y, 2, kd, ix, N);
        double val = H.one(r, p);
        for (int k : oc) val += H.v(r, k, p, k) - H.v(r, k, k, p);
        o.push_back({Key{y.w[0], y.w[1]}, sg * val});
      }
    } else {
      const int p = oc[pairs[t - no].first], q = oc[pairs[t - no].second];
      for (size_t u = 0; u < vi.size(); ++u)
        for (size_t w = u + 1; w < vi.size(); ++w) {
          int r = vi[u], s2 = vi[w];
          int sp = (p >= N) + (q >= N), sr = (r >= N) + (s2 >= N);
          if (sp != sr) continue;
          Occ y = x;
          const char kd[4] = {'c', 'c', 'a', 'a'};
          const int ix[4] = {r, s2, q, p};
          int sg = apply_ops(y, 4, kd, ix, N);
          double val = H.v(r, s2, p, q) - H.v(r, s2, q, p);
          o.push_back({Key{y.w[0], y.w[1]}, sg * val});
        }
    }
  }
  out.clear();
  out.push_back({key, diag_entry(H, x)});
  for (auto& v : piece) out.insert(out.end(), v.begin(), v.end());
}

int oracle_cd_run_mt(int N, const double* h, const double* eri, int ninit, const uint64_t* init_a,
                     const uint64_t* init_b, const double* init_c, double tau, int64_t max_steps,
                     double theta, double dx_tol, int threads, double* traj_E, uint64_t* traj_a,
                     uint64_t* traj_b, double* traj_eta, int64_t* steps_done, double* mu_out,
                     double* alpha_out, int64_t* nstored, int64_t* elements) {
  if (N < 1 || N > 64 || ninit < 1 || threads < 1) return -1;
  Ham H{N, h, eri};
  std::unordered_map<Key, Val, KeyHash> wf;
  wf.reserve(1 << 16);
  std::vector<Elem> col;
  std::vector<Key> cand;
  int64_t nelem = 0;
  for (int t = 0; t < ninit; ++t) wf[Key{init_a[t], init_b[t]}].c += init_c[t];
  for (int t = 0; t < ninit; ++t) {
    Key D{init_a[t], init_b[t]};
    column(H, D, col);
    for (const Elem& e : col) {
      if (e.v == 0.0) continue;
      wf[e.k].b += init_c[t] * e.v;
      cand.push_back(e.k);
    }
  }
  std::sort(cand.begin(), cand.end(), key_less);
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  __float128 mu = 0, alpha = 0;
  for (auto& kv : wf) {
    mu += (__float128)kv.second.c * kv.second.c;
    alpha += (__float128)kv.second.c * kv.second.b;
  }
  std::vector<double> prod, delta;
  std::vector<Val*> node;
  std::vector<char> insert;
  double d = 0.0;
  int64_t step = 0;
  for (; step < max_steps; ++step) {
    const double mud = (double)mu;
    // selection: per-thread best under the total order (g desc, key asc), then joined
    Key best{0, 0};
    double gbest = -1.0;
#pragma omp parallel num_threads(threads)
    {
      Key lb{0, 0};
      double lg = -1.0;
#pragma omp for schedule(static)
      for (int64_t t = 0; t < (int64_t)cand.size(); ++t) {
        const Key& k = cand[t];
        auto it = wf.find(k);
        double c = it == wf.end() ? 0.0 : it->second.c;
        double b = it == wf.end() ? 0.0 : it->second.b;
        double g = fabs(4.0 * b + 4.0 * mud * c);
        if (g > lg || (g == lg && key_less(k, lb))) {
          lb = k;
          lg = g;
        }
      }
#pragma omp critical
      {
        if (lg > gbest || (lg == gbest && key_less(lb, best))) {
          best = lb;
          gbest = lg;
        }
      }
    }
    Key I = best;
    Val& vi = wf[I];
    double ci = vi.c, bi = vi.b;
    double Hii = diag_entry(H, Occ{{I.a, I.b}});
    double eta = line_search(4.0 * bi + 4.0 * mud * ci, 2.0 * Hii + 4.0 * ci * ci + 2.0 * mud, 4.0 * ci);
    vi.c = ci + eta;
    column_mt(H, I, col, threads);
    nelem += (int64_t)col.size();
    const int64_t n = (int64_t)col.size();
    prod.assign(n, 0.0);
    delta.assign(n, 0.0);
    node.assign(n, nullptr);
    insert.assign(n, 0);
    // lookups and updates of existing entries (one writer per entry)
#pragma omp parallel for schedule(static) num_threads(threads)
    for (int64_t t = 1; t < n; ++t) {
      const Elem& e = col[t];
      if (e.v == 0.0) continue;
      const double dl = eta * e.v;
      auto it = wf.find(e.k);
      const double cj = it == wf.end() ? 0.0 : it->second.c;
      if (cj != 0.0 || fabs(dl) >= tau) {
        if (it == wf.end()) {
          insert[t] = 1;
          delta[t] = dl;
        } else {
          it->second.b += dl;
        }
      }
      prod[t] = e.v * cj;
    }
    cand.clear();
    double recalc = col[0].v * (ci + eta);
    cand.push_back(I);
    for (int64_t t = 1; t < n; ++t) {
      const Elem& e = col[t];
      if (e.v == 0.0) continue;
      cand.push_back(e.k);
      if (insert[t]) wf.emplace(e.k, Val{}).first->second.b += delta[t];
      recalc += prod[t];
    }
    Val& vi2 = wf[I];
    vi2.b = recalc;
    mu += 2 * (__float128)eta * ci + (__float128)eta * eta;
    alpha += 2 * (__float128)eta * bi + (__float128)eta * eta * Hii;
    if (mu <= 0) return -2;
    d = step == 0 ? fabs(eta) : theta * d + (1.0 - theta) * fabs(eta);
    if (traj_E) traj_E[step] = (double)(alpha / mu);
    if (traj_a) traj_a[step] = I.a;
    if (traj_b) traj_b[step] = I.b;
    if (traj_eta) traj_eta[step] = eta;
    if (d < dx_tol) {
      ++step;
      break;
    }
  }
  *steps_done = step;
  *mu_out = (double)mu;
  *alpha_out = (double)alpha;
  *nstored = (int64_t)wf.size();
  *elements = nelem;
  return 0;
}

}  // extern "C"
