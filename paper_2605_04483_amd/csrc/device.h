// Device building blocks of the coordinate-descent FCI hot path (gfx950).
//
//   * determinant keys: {alpha, beta} 64-bit occupation strings;
//   * open-addressing hash table of 32-byte slots {key_alpha, key_beta, c, b}
//     with a claim/publish insert (64-bit CAS on the alpha word, then a
//     release store of the beta word);
//   * Slater-Condon entries (paper Sec. 2.3, eq. (entry)) evaluated from the
//     occupied/virtual lists of the column's determinant, fermionic phases by
//     popcount over the orbitals strictly between the moved indices;
//   * double-double accumulation for mu = c.c and alpha = c.Hc (the paper keeps
//     them in quad precision, Sec. 4.1.2), Dekker/Knuth two-sum and two-prod;
//   * the exact line search of the quartic (Sec. 3.1 eq. (choose-alpha),
//     Appendix A): Cardano per Nickalls, Newton polish, lowest critical value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdfci {

constexpr uint64_t kEmpty = ~0ull;    // alpha word of a free slot
constexpr uint64_t kPending = ~0ull;  // beta word not yet published
constexpr int kMaxProbe = 4096;       // probe sequence bound (then TABLE_FULL)
constexpr int kMaxOrb = 63;

// error flags raised from device code (ORed into the control block)
constexpr int kErrTableFull = 1;
constexpr int kErrBarrier = 2;
constexpr int kErrPublish = 4;
constexpr int kErrNumeric = 8;
constexpr int kErrSelect = 16;  // a selection's bound held fewer than k distinct determinants

struct alignas(32) Slot {
  uint64_t ka, kb;
  double c, b;
};

// Hamiltonian view.  eri is the packed 8-fold-symmetric chemist tensor (see
// ERI below); the full N^4 tensor is kept separately where it is contracted.
struct Ham {
  int N, na, nb;
  const double* __restrict__ h;
  const double* __restrict__ eri;
  // jk[((r*N + p)*N + k)*2 + {0,1}] = {(rp|kk), (rk|kp)}: the Coulomb and
  // exchange integrals a single excitation p -> r sums over occupied k, laid
  // out contiguously in k so one excitation reads one short row
  const double* __restrict__ jk;
};

// ---------------------------------------------------------------- bits

__device__ __forceinline__ int popc(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ int ctz(uint64_t x) { return __ffsll((unsigned long long)x) - 1; }
// bits strictly between p and r (p != r)
__device__ __forceinline__ uint64_t between(int p, int r) {
  int lo = p < r ? p : r, hi = p < r ? r : p;
  return ((1ull << hi) - 1ull) & ~((2ull << lo) - 1ull);
}
__device__ __forceinline__ int parity_between(uint64_t s, int p, int r) {
  return popc(s & between(p, r)) & 1;
}

__device__ __forceinline__ uint64_t hash_key(uint64_t a, uint64_t b) {
  // splitmix64 finaliser over a mix of both words
  uint64_t x = a ^ (b * 0x9E3779B97F4A7C15ull) ^ (b >> 29);
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

__device__ __forceinline__ bool key_less(uint64_t a1, uint64_t b1, uint64_t a2, uint64_t b2) {
  return b1 != b2 ? b1 < b2 : a1 < a2;
}

// ---------------------------------------------------------------- atomics

__device__ __forceinline__ uint64_t ld_acq(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double atomic_add_f64(double* p, double v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Coherent (agent-scope) accesses for data that several workgroups touch inside
// one persistent launch.  They are serviced at the device coherence point, so
// no L2 write-back / invalidate is needed at a device-wide barrier and the
// read-only integrals stay L2-resident across iterations.
__device__ __forceinline__ uint64_t ld_co(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_co(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld_co(const int64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_co(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_co(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_co(int64_t* p, int64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A slot's four words, fetched together.
struct SlotVal {
  uint64_t ka, kb;
  double c, b;
};
__device__ __forceinline__ SlotVal slot_load(const Slot* s) {
  SlotVal v;
  v.ka = ld_co(&s->ka);
  v.kb = ld_co(&s->kb);
  v.c = ld_co(&s->c);
  v.b = ld_co(&s->b);
  return v;
}

// ---------------------------------------------------------------- hash table

// Find key; returns slot or -1 and, when found, the slot's words in *val.
// *probes receives the probe count.
__device__ inline int64_t table_find(const Slot* __restrict__ T, uint64_t mask, uint64_t a,
                                     uint64_t b, int* probes, SlotVal* val) {
  uint64_t idx = hash_key(a, b) & mask;
  for (int n = 0; n < kMaxProbe; ++n) {
    SlotVal v = slot_load(&T[idx]);
    if (v.ka == kEmpty) {
      *probes = n + 1;
      return -1;
    }
    if (v.ka == a) {
      if (v.kb == kPending) {
        int spin = 0;
        do {
          v.kb = ld_co(&T[idx].kb);
        } while (v.kb == kPending && ++spin < (1 << 20));
        // c and b are meaningful once the beta word is published
        v.c = ld_co(&T[idx].c);
        v.b = ld_co(&T[idx].b);
      }
      if (v.kb == b) {
        *probes = n + 1;
        *val = v;
        return (int64_t)idx;
      }
    }
    idx = (idx + 1) & mask;
  }
  *probes = kMaxProbe;
  return -1;
}

// table_find with the first probe's slot already loaded (issued early by the
// caller, so its latency runs under other work); same result as table_find
__device__ inline int64_t table_find_from(const Slot* __restrict__ T, uint64_t mask, uint64_t a, uint64_t b,
                                          SlotVal first, int* probes, SlotVal* val) {
  uint64_t idx = hash_key(a, b) & mask;
  for (int n = 0; n < kMaxProbe; ++n) {
    SlotVal v = n == 0 ? first : slot_load(&T[idx]);
    if (v.ka == kEmpty) {
      *probes = n + 1;
      return -1;
    }
    if (v.ka == a) {
      if (v.kb == kPending) {
        int spin = 0;
        do {
          v.kb = ld_co(&T[idx].kb);
        } while (v.kb == kPending && ++spin < (1 << 20));
        v.c = ld_co(&T[idx].c);
        v.b = ld_co(&T[idx].b);
      }
      if (v.kb == b) {
        *probes = n + 1;
        *val = v;
        return (int64_t)idx;
      }
    }
    idx = (idx + 1) & mask;
  }
  *probes = kMaxProbe;
  return -1;
}

// Find or insert; returns slot, or -1 on probe overflow / publish timeout
// (*err gets the flag).  *inserted = 1 if this call claimed the slot.  The
// slot's c and b are returned in *val (zeros for a fresh slot).
__device__ inline int64_t table_upsert(Slot* __restrict__ T, uint64_t mask, uint64_t a, uint64_t b,
                                       int* inserted, int* probes, int* err, SlotVal* val) {
  uint64_t idx = hash_key(a, b) & mask;
  *inserted = 0;
  for (int n = 0; n < kMaxProbe; ++n) {
    SlotVal v = slot_load(&T[idx]);
    uint64_t ka = v.ka;
    if (ka == kEmpty) {
      uint64_t old = atomicCAS((unsigned long long*)&T[idx].ka, (unsigned long long)kEmpty,
                               (unsigned long long)a);
      if (old == kEmpty) {
        st_co(&T[idx].kb, b);
        *inserted = 1;
        *probes = n + 1;
        *val = SlotVal{a, b, 0.0, 0.0};
        return (int64_t)idx;
      }
      ka = old;
      v.kb = ld_co(&T[idx].kb);
      v.c = ld_co(&T[idx].c);
      v.b = ld_co(&T[idx].b);
    }
    if (ka == a) {
      uint64_t kb = v.kb;
      if (kb == kPending) {
        int spin = 0;
        do {
          kb = ld_co(&T[idx].kb);
        } while (kb == kPending && ++spin < (1 << 20));
        if (kb == kPending) {
          *err |= kErrPublish;
          return -1;
        }
        v.c = ld_co(&T[idx].c);
        v.b = ld_co(&T[idx].b);
      }
      if (kb == b) {
        *probes = n + 1;
        v.ka = a;
        v.kb = b;
        *val = v;
        return (int64_t)idx;
      }
    }
    idx = (idx + 1) & mask;
  }
  *probes = kMaxProbe;
  *err |= kErrTableFull;
  return -1;
}

// table_upsert for a key whose find has just ended at the empty slot idx0
// after nprev occupied slots: the claim is tried there at once, with no reload
// and no second walk of the chain before it (those slots held other keys, and
// within an iteration no other lane inserts this key).  If another key took
// idx0 meanwhile, the walk continues from there as in table_upsert.
__device__ inline int64_t table_upsert_at(Slot* __restrict__ T, uint64_t mask, uint64_t a, uint64_t b,
                                          uint64_t idx0, int nprev, int* inserted, int* probes, int* err,
                                          SlotVal* val) {
  uint64_t idx = idx0;
  *inserted = 0;
  for (int n = nprev; n < kMaxProbe; ++n) {
    SlotVal v;
    if (n == nprev) {
      v = SlotVal{kEmpty, 0, 0.0, 0.0};
    } else {
      v = slot_load(&T[idx]);
    }
    uint64_t ka = v.ka;
    if (ka == kEmpty) {
      uint64_t old = atomicCAS((unsigned long long*)&T[idx].ka, (unsigned long long)kEmpty,
                               (unsigned long long)a);
      if (old == kEmpty) {
        st_co(&T[idx].kb, b);
        *inserted = 1;
        *probes = n + 1;
        *val = SlotVal{a, b, 0.0, 0.0};
        return (int64_t)idx;
      }
      ka = old;
      v.kb = ld_co(&T[idx].kb);
      v.c = ld_co(&T[idx].c);
      v.b = ld_co(&T[idx].b);
    }
    if (ka == a) {
      uint64_t kb = v.kb;
      if (kb == kPending) {
        int spin = 0;
        do {
          kb = ld_co(&T[idx].kb);
        } while (kb == kPending && ++spin < (1 << 20));
        if (kb == kPending) {
          *err |= kErrPublish;
          return -1;
        }
        v.c = ld_co(&T[idx].c);
        v.b = ld_co(&T[idx].b);
      }
      if (kb == b) {
        *probes = n + 1;
        v.ka = a;
        v.kb = b;
        *val = v;
        return (int64_t)idx;
      }
    }
    idx = (idx + 1) & mask;
  }
  *probes = kMaxProbe;
  *err |= kErrTableFull;
  return -1;
}

// ---------------------------------------------------------------- double-double

struct dd {
  double hi, lo;
};
__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  double lo = s.lo + x.lo + y.lo;
  return two_sum(s.hi, lo);
}
__device__ __forceinline__ dd dd_mul_d(dd x, double y) {
  dd p = two_prod(x.hi, y);
  double lo = p.lo + x.lo * y;
  return two_sum(p.hi, lo);
}
__device__ __forceinline__ dd dd_mul(dd x, dd y) {
  dd p = two_prod(x.hi, y.hi);
  double lo = p.lo + (x.hi * y.lo + x.lo * y.hi);
  return two_sum(p.hi, lo);
}
__device__ __forceinline__ double dd_val(dd x) { return x.hi + x.lo; }

// workgroup sum (any power-of-two size up to 1024), fixed order
__device__ inline double wg_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(v, off);
    v = (lane & off) ? (o + v) : (v + o);
  }
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  __syncthreads();
  return s;
}

__device__ inline dd wg_sum_dd(dd v, double* scratch) {
  double hi = wg_sum(v.hi, scratch);
  double lo = wg_sum(v.lo, scratch);
  return two_sum(hi, lo);
}

// ---------------------------------------------------------------- line search

__device__ __forceinline__ double quartic(double e, double v1, double v2, double v3) {
  return ((e + v3) * e + v2) * e * e + v1 * e;
}

// argmin of h(eta) = eta^4 + v3 eta^3 + v2 eta^2 + v1 eta: real roots of
// h'(eta) = 4 eta^3 + 3 v3 eta^2 + 2 v2 eta + v1 by Cardano's method, each
// polished by Newton's iteration, lowest h wins (ties: smaller |eta|).
__device__ inline double line_search(double v1, double v2, double v3) {
  // normalised cubic eta^3 + B eta^2 + C eta + D, depressed via eta = x - B/3
  const double B = 0.75 * v3, C = 0.5 * v2, D = 0.25 * v1;
  const double p = C - B * B / 3.0;
  const double q = (2.0 * B * B * B) / 27.0 - B * C / 3.0 + D;
  const double disc = 0.25 * q * q + (p * p * p) / 27.0;
  // Newton's iteration on h'; a correction of a few ulp means converged
  auto polish = [&](double x) {
    for (int it = 0; it < 8; ++it) {
      double f = ((4.0 * x + 3.0 * v3) * x + 2.0 * v2) * x + v1;
      double fp = (12.0 * x + 6.0 * v3) * x + 2.0 * v2;
      if (fp == 0.0) break;
      double dx = f / fp;
      x -= dx;
      if (fabs(dx) <= 4.5e-16 * fabs(x)) break;
    }
    return x;
  };
  if (disc > 0.0 || p == 0.0) {
    double r0;
    if (p == 0.0 && disc <= 0.0) {
      r0 = -B / 3.0;
    } else {
      double sd = sqrt(disc);
      r0 = cbrt(-0.5 * q + sd) + cbrt(-0.5 * q - sd) - B / 3.0;
    }
    return polish(r0);
  }
  const double m = 2.0 * sqrt(-p / 3.0);
  double arg = (1.5 * q / p) * sqrt(-3.0 / p);
  arg = fmin(1.0, fmax(-1.0, arg));
  // trigonometric form: x_k = m cos(th - 2 pi k / 3), th = acos(arg) / 3; the
  // k = 1, 2 roots follow from cos th and sin th by the angle-sum identity
  const double th = acos(arg) / 3.0;
  const double ct = cos(th), st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double half_sqrt3 = 0.86602540378443864676;
  double best = polish(m * ct - B / 3.0);
  double bh = quartic(best, v1, v2, v3);
  double x1 = polish(m * (-0.5 * ct + half_sqrt3 * st) - B / 3.0);
  double h1 = quartic(x1, v1, v2, v3);
  if (h1 < bh || (h1 == bh && fabs(x1) < fabs(best))) {
    best = x1;
    bh = h1;
  }
  double x2 = polish(m * (-0.5 * ct - half_sqrt3 * st) - B / 3.0);
  double h2 = quartic(x2, v1, v2, v3);
  if (h2 < bh || (h2 == bh && fabs(x2) < fabs(best))) best = x2;
  return best;
}

// ---------------------------------------------------------------- Slater-Condon

// (pq|rs) from the packed tensor: one value per orbit of the 8-fold symmetry
// (pq|rs) = (qp|rs) = (pq|sr) = (rs|pq) = ..., at the canonical position of
// the ordered pairs pq >= rs with p >= q, r >= s.  N(N+1)/2 (N(N+1)/2 + 1) / 2
// values: 1.78 MB at 36 orbitals, small enough to stay in one XCD's L2.
__device__ __forceinline__ int pair_index(int p, int q) {
  return p >= q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p;
}
__device__ __forceinline__ int64_t eri8_index(int p, int q, int r, int s) {
  const int64_t pq = pair_index(p, q), rs = pair_index(r, s);
  return pq >= rs ? pq * (pq + 1) / 2 + rs : rs * (rs + 1) / 2 + pq;
}
__device__ __forceinline__ double ERI(const Ham& H, int p, int q, int r, int s) {
  return H.eri[eri8_index(p, q, r, s)];
}

// Occupied / virtual orbital lists of the column's determinant.
struct Lists {
  int8_t oa[64], va[64], ob[64], vb[64];
  int na, nva, nb, nvb;
};

// Same lists built by a workgroup: thread p places orbital p by a popcount of
// the lower bits.  Threads 0..N-1 must take part; a barrier must follow.
__device__ inline void make_lists_block(uint64_t a, uint64_t b, int N, Lists& L) {
  const int t = threadIdx.x;
  if (t < N) {
    const uint64_t below = (1ull << t) - 1ull;
    const int ia = popc(a & below), ib = popc(b & below);
    if ((a >> t) & 1) L.oa[ia] = (int8_t)t;
    else L.va[t - ia] = (int8_t)t;
    if ((b >> t) & 1) L.ob[ib] = (int8_t)t;
    else L.vb[t - ib] = (int8_t)t;
  }
  if (t == 0) {
    L.na = popc(a);
    L.nva = N - L.na;
    L.nb = popc(b);
    L.nvb = N - L.nb;
  }
}

__device__ inline void make_lists_serial(uint64_t a, uint64_t b, int N, Lists& L) {
  int i = 0, j = 0;
  for (int p = 0; p < N; ++p) {
    if ((a >> p) & 1) L.oa[i++] = (int8_t)p;
    else L.va[j++] = (int8_t)p;
  }
  L.na = i;
  L.nva = j;
  i = j = 0;
  for (int p = 0; p < N; ++p) {
    if ((b >> p) & 1) L.ob[i++] = (int8_t)p;
    else L.vb[j++] = (int8_t)p;
  }
  L.nb = i;
  L.nvb = j;
}

// number of entries of get_column (diagonal included)
__host__ __device__ inline int64_t column_count(int N, int na, int nb) {
  int64_t va = N - na, vb = N - nb;
  int64_t ca = (int64_t)na * (na - 1) / 2, cb = (int64_t)nb * (nb - 1) / 2;
  int64_t cva = va * (va - 1) / 2, cvb = vb * (vb - 1) / 2;
  return 1 + na * va + nb * vb + ca * cva + cb * cvb + (int64_t)na * va * nb * vb;
}

// decode t in [0, n(n-1)/2) into i < j with t = j(j-1)/2 + i
__device__ __forceinline__ void pair_decode(int t, int& i, int& j) {
  int jj = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
  while (jj * (jj - 1) / 2 > t) --jj;
  while ((jj + 1) * jj / 2 <= t) ++jj;
  j = jj;
  i = t - jj * (jj - 1) / 2;
}

// H_DD (eq. (entry), diagonal case), serial over the occupied lists
__device__ inline double diag_serial(const Ham& H, const Lists& L) {
  double e = 0.0;
  for (int i = 0; i < L.na; ++i) e += H.h[L.oa[i] * H.N + L.oa[i]];
  for (int i = 0; i < L.nb; ++i) e += H.h[L.ob[i] * H.N + L.ob[i]];
  double two = 0.0;
  for (int i = 0; i < L.na; ++i)
    for (int j = 0; j < L.na; ++j) {
      int p = L.oa[i], q = L.oa[j];
      two += ERI(H, p, p, q, q) - ERI(H, p, q, q, p);
    }
  for (int i = 0; i < L.nb; ++i)
    for (int j = 0; j < L.nb; ++j) {
      int p = L.ob[i], q = L.ob[j];
      two += ERI(H, p, p, q, q) - ERI(H, p, q, q, p);
    }
  double ab = 0.0;
  for (int i = 0; i < L.na; ++i)
    for (int j = 0; j < L.nb; ++j) ab += ERI(H, L.oa[i], L.oa[i], L.ob[j], L.ob[j]);
  return e + 0.5 * two + ab;
}

// Term t of H_DD split into independent pieces so a workgroup can share them:
// one-body h_pp, same-spin pairs 1/2[(pp|qq) - (pq|qp)], opposite-spin (pp|qq).
__host__ __device__ inline int diag_terms(const Lists& L) {
  return L.na + L.nb + L.na * L.na + L.nb * L.nb + L.na * L.nb;
}
__device__ inline double diag_term(const Ham& H, const Lists& L, int t) {
  if (t < L.na) return H.h[L.oa[t] * H.N + L.oa[t]];
  t -= L.na;
  if (t < L.nb) return H.h[L.ob[t] * H.N + L.ob[t]];
  t -= L.nb;
  if (t < L.na * L.na) {
    int p = L.oa[t / L.na], q = L.oa[t % L.na];
    return 0.5 * (ERI(H, p, p, q, q) - ERI(H, p, q, q, p));
  }
  t -= L.na * L.na;
  if (t < L.nb * L.nb) {
    int p = L.ob[t / L.nb], q = L.ob[t % L.nb];
    return 0.5 * (ERI(H, p, p, q, q) - ERI(H, p, q, q, p));
  }
  t -= L.nb * L.nb;
  return ERI(H, L.oa[t / L.nb], L.oa[t / L.nb], L.ob[t % L.nb], L.ob[t % L.nb]);
}

// diag_term(t) as f (x - y) with its integrals loaded and the arithmetic left
// to the caller (y = 0 and f = 1 where diag_term has no exchange part: the
// same value bit for bit)
struct DiagLoad {
  double x, y, f;
};

__device__ inline DiagLoad diag_term_load(const Ham& H, const Lists& L, int t) {
  if (t < L.na) return DiagLoad{H.h[L.oa[t] * H.N + L.oa[t]], 0.0, 1.0};
  t -= L.na;
  if (t < L.nb) return DiagLoad{H.h[L.ob[t] * H.N + L.ob[t]], 0.0, 1.0};
  t -= L.nb;
  if (t < L.na * L.na) {
    int p = L.oa[t / L.na], q = L.oa[t % L.na];
    return DiagLoad{ERI(H, p, p, q, q), ERI(H, p, q, q, p), 0.5};
  }
  t -= L.na * L.na;
  if (t < L.nb * L.nb) {
    int p = L.ob[t / L.nb], q = L.ob[t % L.nb];
    return DiagLoad{ERI(H, p, p, q, q), ERI(H, p, q, q, p), 0.5};
  }
  t -= L.nb * L.nb;
  return DiagLoad{ERI(H, L.oa[t / L.nb], L.oa[t / L.nb], L.ob[t % L.nb], L.ob[t % L.nb]), 0.0, 1.0};
}

// single p -> r within spin sigma (same: occupied list of that spin, other:
// the opposite spin's occupied list); value before the phase
__device__ inline double single_value(const Ham& H, int p, int r, const int8_t* same, int ns,
                                      const int8_t* other, int no) {
  const double* row = H.jk + (size_t)(r * H.N + p) * H.N * 2;
  double v = H.h[r * H.N + p];
  for (int k = 0; k < ns; ++k) {
    int kk = same[k];
    v += row[2 * kk] - row[2 * kk + 1];
  }
  for (int k = 0; k < no; ++k) v += row[2 * other[k]];
  return v;
}

// Excitation of entry e of get_column(D), in the library's enumeration order:
//   0                      diagonal                       type 0
//   alpha singles          na*va   (occupied index major)  type 1: p -> r
//   beta singles           nb*vb                           type 2: p -> r
//   alpha-alpha doubles    C(na,2)*C(va,2) (occupied pair major) type 3: p<q -> r<s
//   beta-beta doubles      C(nb,2)*C(vb,2)                 type 4: p<q -> r<s
//   alpha-beta doubles     na*va*nb*vb (alpha single major) type 5: p->r alpha, q->s beta
// The fermionic phase `neg` is that of a+_r a_p (singles) or a+_r a+_s a_q a_p
// (doubles) on D; the excited key is written to (oa, ob).  Column sizes stay
// below 2^31 for at most 63 orbitals, so the decoding uses 32-bit arithmetic.
struct Excitation {
  int type, p, q, r, s, neg;
};

__device__ inline Excitation decode_excitation(const Lists& L, uint64_t a, uint64_t b, uint32_t e,
                                               uint64_t* oa, uint64_t* ob) {
  Excitation x{0, 0, 0, 0, 0, 0};
  *oa = a;
  *ob = b;
  if (e == 0) return x;
  e -= 1;
  const uint32_t sa = (uint32_t)(L.na * L.nva);
  if (e < sa) {
    x.type = 1;
    x.p = L.oa[e / L.nva];
    x.r = L.va[e % L.nva];
    *oa = a ^ (1ull << x.p) ^ (1ull << x.r);
    x.neg = parity_between(a, x.p, x.r);
    return x;
  }
  e -= sa;
  const uint32_t sb = (uint32_t)(L.nb * L.nvb);
  if (e < sb) {
    x.type = 2;
    x.p = L.ob[e / L.nvb];
    x.r = L.vb[e % L.nvb];
    *ob = b ^ (1ull << x.p) ^ (1ull << x.r);
    x.neg = parity_between(b, x.p, x.r);
    return x;
  }
  e -= sb;
  const uint32_t qa = (uint32_t)(L.nva * (L.nva - 1) / 2);
  const uint32_t daa = (uint32_t)(L.na * (L.na - 1) / 2) * qa;
  if (e < daa) {
    int i, j, u, v;
    pair_decode((int)(e / qa), i, j);
    pair_decode((int)(e % qa), u, v);
    x.type = 3;
    x.p = L.oa[i];
    x.q = L.oa[j];
    x.r = L.va[u];
    x.s = L.va[v];
    const uint64_t a1 = a ^ (1ull << x.p) ^ (1ull << x.r);
    x.neg = parity_between(a, x.p, x.r) ^ parity_between(a1, x.q, x.s);
    *oa = a1 ^ (1ull << x.q) ^ (1ull << x.s);
    return x;
  }
  e -= daa;
  const uint32_t qb = (uint32_t)(L.nvb * (L.nvb - 1) / 2);
  const uint32_t dbb = (uint32_t)(L.nb * (L.nb - 1) / 2) * qb;
  if (e < dbb) {
    int i, j, u, v;
    pair_decode((int)(e / qb), i, j);
    pair_decode((int)(e % qb), u, v);
    x.type = 4;
    x.p = L.ob[i];
    x.q = L.ob[j];
    x.r = L.vb[u];
    x.s = L.vb[v];
    const uint64_t b1 = b ^ (1ull << x.p) ^ (1ull << x.r);
    x.neg = parity_between(b, x.p, x.r) ^ parity_between(b1, x.q, x.s);
    *ob = b1 ^ (1ull << x.q) ^ (1ull << x.s);
    return x;
  }
  e -= dbb;
  const uint32_t sbb = (uint32_t)(L.nb * L.nvb);
  const uint32_t ia = e / sbb, ib = e % sbb;
  x.type = 5;
  x.p = L.oa[ia / L.nva];
  x.r = L.va[ia % L.nva];
  x.q = L.ob[ib / L.nvb];
  x.s = L.vb[ib % L.nvb];
  *oa = a ^ (1ull << x.p) ^ (1ull << x.r);
  *ob = b ^ (1ull << x.q) ^ (1ull << x.s);
  x.neg = parity_between(a, x.p, x.r) ^ parity_between(b, x.q, x.s);
  return x;
}

// Entry e of get_column(D): writes the excited key and returns H_{D',D}
// (eq. (entry)); `diag` supplies H_DD for e = 0.
__device__ inline double column_entry(const Ham& H, const Lists& L, uint64_t a, uint64_t b,
                                      int64_t e, double diag, uint64_t* oa_out, uint64_t* ob_out) {
  const Excitation x = decode_excitation(L, a, b, (uint32_t)e, oa_out, ob_out);
  double v;
  switch (x.type) {
    case 0:
      return diag;
    case 1:
      v = single_value(H, x.p, x.r, L.oa, L.na, L.ob, L.nb);
      break;
    case 2:
      v = single_value(H, x.p, x.r, L.ob, L.nb, L.oa, L.na);
      break;
    case 3:
    case 4:
      v = ERI(H, x.r, x.p, x.s, x.q) - ERI(H, x.r, x.q, x.s, x.p);
      break;
    default:
      v = ERI(H, x.r, x.p, x.s, x.q);
      break;
  }
  return x.neg ? -v : v;
}

// get_entry: H_{bra,ket} by classifying the difference of the two keys.
__device__ inline double sc_entry(const Ham& H, uint64_t bra_a, uint64_t bra_b, uint64_t ket_a,
                                  uint64_t ket_b, const Lists& Lket, double diag_ket) {
  uint64_t da = bra_a ^ ket_a, db = bra_b ^ ket_b;
  int na = popc(da), nb = popc(db);
  if (na + nb == 0) return diag_ket;
  if (na + nb > 4) return 0.0;
  if (na == 2 && nb == 0) {
    int p = ctz(da & ket_a), r = ctz(da & bra_a);
    double v = single_value(H, p, r, Lket.oa, Lket.na, Lket.ob, Lket.nb);
    return parity_between(ket_a, p, r) ? -v : v;
  }
  if (na == 0 && nb == 2) {
    int p = ctz(db & ket_b), r = ctz(db & bra_b);
    double v = single_value(H, p, r, Lket.ob, Lket.nb, Lket.oa, Lket.na);
    return parity_between(ket_b, p, r) ? -v : v;
  }
  if (na == 4 || nb == 4) {
    uint64_t s_ket = na == 4 ? ket_a : ket_b, d = na == 4 ? da : db;
    uint64_t holes = d & s_ket, parts = d & ~s_ket;
    int p = ctz(holes), q = ctz(holes & (holes - 1));
    int r = ctz(parts), s = ctz(parts & (parts - 1));
    uint64_t s1 = s_ket ^ (1ull << p) ^ (1ull << r);
    int sg = parity_between(s_ket, p, r) ^ parity_between(s1, q, s);
    double v = ERI(H, r, p, s, q) - ERI(H, r, q, s, p);
    return sg ? -v : v;
  }
  // alpha-beta double
  int p = ctz(da & ket_a), r = ctz(da & bra_a);
  int q = ctz(db & ket_b), s = ctz(db & bra_b);
  double v = ERI(H, r, p, s, q);
  return (parity_between(ket_a, p, r) ^ parity_between(ket_b, q, s)) ? -v : v;
}

}  // namespace cdfci
