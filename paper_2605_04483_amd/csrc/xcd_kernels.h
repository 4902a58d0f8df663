// Coordinate descent for several low-lying states, xCDFCI (paper Sec. 3.3,
// Algorithm 3; line search in Appendix A), device side.  Included into
// cdfci.hip inside its kernel namespace.
//
// C has n = K + 1 columns (one per state) and is stored by rows: the table
// holds, per determinant j, its key and the rows C_j and B_j (B = H C).  The
// n x n matrices S = C^T C and Q = C^T H C are maintained in double-double.
// With G = 4B + 4CS one iteration takes i = argmax ||G_j||_inf over the
// column of the previous coordinate (plus that coordinate), the step
// C <- C + eta e_i g with g = G_i and eta the minimiser of
// h(eta) = f(C + eta e_i g) - f(C) = w4 eta^4 + w3 eta^3 + w2 eta^2 + w1 eta,
//   w1 = |g|^2, w2 = 2 H_ii |g|^2 + 2 (C_i.g)^2 + 2 |C_i|^2 |g|^2 + 2 g S g^T,
//   w3 = 4 |g|^2 (C_i.g), w4 = |g|^4
// (the slope w1 = <G, e_i g> = |g|^2; the appendix prints 4|g|^2, which the
// other coefficients and the one-state case contradict), then
// S += eta (C_i^T g + g^T C_i) + eta^2 g^T g, Q += eta (B_i^T g + g^T B_i)
// + eta^2 H_ii g^T g (outer products, pre-step rows), B_j += eta H_ji g over
// the column (compression: iff C_j != 0 or |eta H_ji| |g|_inf >= tau), and
// B_i = sum_j H_ji C_j recomputed.  An optional shift sigma replaces H by
// H - sigma I (every diagonal element).
//
// The iteration kernel runs persistently (one cooperative launch for a
// call's iterations, one device-wide barrier each); see k_xiter below.

constexpr int kXMax = 8;  // states per context (K + 1)

struct XKey {
  uint64_t ka, kb;  // the Slot key protocol: claim ka by CAS, then publish kb
};

struct XCtl {
  double S_hi[kXMax * kXMax], S_lo[kXMax * kXMax];  // double-double, n x n row-major
  double Q_hi[kXMax * kXMax], Q_lo[kXMax * kXMax];
  uint64_t ia, ib;  // coordinate of the coming iteration
  int64_t islot;
  double d;  // damped step accumulator
  double shift;
  int64_t steps;
  int64_t steps_this_call;
  unsigned long long occupied, inserts;
  int error, stopped;
  int n, max_probe;
  unsigned arrive;
  int pad;
};

struct XPartial {
  double gmax;
  uint64_t ka, kb;
  int64_t slot;
  double rec[kXMax];  // sum of H_ji C_j over the workgroup's entries
  int64_t inserts;
  int64_t err;  // error bits
};

// Momentum-space Hubbard model (the Hubbard model of Sec. 2.2 in the Bloch
// orbitals of the periodic lattice, Sec. 4.1.1 HubbardK): orbital k is the
// row-major index of a momentum vector, eps[k] its one-body energy, and the
// on-site term becomes (U/L) sum_{k,p,q} a+_{k+q up} a_{k up} a+_{p-q dn} a_{p dn}.
// A column therefore holds the diagonal, sum eps over the occupied orbitals
// + (U/L) n_up n_dn, and the pair moves k -> k+q (up), p -> p-q (down) for
// q != 0 with both targets empty, each (U/L) times the two strings' signs.
struct HamK {
  int L, ndim;
  int dims[3];
  const double* eps;
  double u;  // U / L
};

__device__ __forceinline__ int k_shift(const HamK& K, int k, int q, int sgn) {
  int out = 0, mul = 1;
  for (int d = K.ndim - 1; d >= 0; --d) {
    const int n = K.dims[d];
    const int kd = k % n, qd = q % n;
    k /= n;
    q /= n;
    out += ((kd + sgn * qd + n) % n) * mul;
    mul *= n;
  }
  return out;
}

// (-1)^(electrons of s strictly between orbitals x and y)
__device__ __forceinline__ double between_sign(uint64_t s, int x, int y) {
  const int lo = min(x, y), hi = max(x, y);
  const uint64_t m = ((hi >= 64 ? ~0ull : (1ull << hi)) - 1ull) & ~((2ull << lo) - 1ull);
  return (popc(s & m) & 1) ? -1.0 : 1.0;
}

__host__ __device__ inline int64_t column_count_k(int L, int na, int nb) {
  return 1 + (int64_t)na * nb * (L - 1);
}

// entry e >= 1 of the column of (a, b): 0 when a target is occupied
__device__ inline double column_entry_k(const HamK& K, const Lists& Ls, uint64_t a, uint64_t b, int64_t e,
                                        uint64_t* ja, uint64_t* jb) {
  int64_t t = e - 1;
  const int q = 1 + (int)(t % (K.L - 1));
  t /= (K.L - 1);
  const int ib_i = (int)(t % Ls.nb), ia_i = (int)(t / Ls.nb);
  const int k = Ls.oa[ia_i], p = Ls.ob[ib_i];
  const int kq = k_shift(K, k, q, 1), pq = k_shift(K, p, q, -1);
  *ja = a;
  *jb = b;
  if (((a >> kq) & 1) || ((b >> pq) & 1)) return 0.0;
  *ja = a ^ (1ull << k) ^ (1ull << kq);
  *jb = b ^ (1ull << p) ^ (1ull << pq);
  return K.u * between_sign(a, k, kq) * between_sign(b, p, pq);
}

struct XArgs {
  int64_t nsteps;  // iterations of one launch
  Ham H;
  HamK HK;
  XKey* K;
  double* R;  // rows: slot s -> R[s * 2n .. +n) = C_s, [+n .. +2n) = B_s
  uint64_t mask, max_entries;
  XCtl* x;
  XPartial* parts;
  int64_t n_col;
  double tau, theta, dx_tol;
  double* tr_SQ;  // optional: S and Q after each step (2 n^2 doubles per step)
  uint64_t* tr_a;
  uint64_t* tr_b;
};

// ---------------------------------------------------------------- key table

__device__ inline int64_t xkey_find(const XKey* __restrict__ K, uint64_t mask, uint64_t a, uint64_t b,
                                    int* probes) {
  uint64_t idx = hash_key(a, b) & mask;
  for (int n = 0; n < kMaxProbe; ++n) {
    const uint64_t ka = ld_co(&K[idx].ka);
    if (ka == kEmpty) {
      *probes = n + 1;
      return -1;
    }
    if (ka == a) {
      uint64_t kb = ld_co(&K[idx].kb);
      int spin = 0;
      while (kb == kPending && ++spin < (1 << 20)) kb = ld_co(&K[idx].kb);
      if (kb == b) {
        *probes = n + 1;
        return (int64_t)idx;
      }
    }
    idx = (idx + 1) & mask;
  }
  *probes = kMaxProbe;
  return -1;
}

// find or claim; *inserted = 1 for a fresh slot (rows still zero)
__device__ inline int64_t xkey_upsert(XKey* __restrict__ K, uint64_t mask, uint64_t a, uint64_t b,
                                      int* inserted, int* probes, int* err) {
  uint64_t idx = hash_key(a, b) & mask;
  *inserted = 0;
  for (int n = 0; n < kMaxProbe; ++n) {
    uint64_t ka = ld_co(&K[idx].ka);
    if (ka == kEmpty) {
      const uint64_t old = atomicCAS((unsigned long long*)&K[idx].ka, (unsigned long long)kEmpty,
                                     (unsigned long long)a);
      if (old == kEmpty) {
        st_co(&K[idx].kb, b);
        *inserted = 1;
        *probes = n + 1;
        return (int64_t)idx;
      }
      ka = old;
    }
    if (ka == a) {
      uint64_t kb = ld_co(&K[idx].kb);
      int spin = 0;
      while (kb == kPending && ++spin < (1 << 20)) kb = ld_co(&K[idx].kb);
      if (kb == kPending) {
        *err |= kErrPublish;
        return -1;
      }
      if (kb == b) {
        *probes = n + 1;
        return (int64_t)idx;
      }
    }
    idx = (idx + 1) & mask;
  }
  *probes = kMaxProbe;
  *err |= kErrTableFull;
  return -1;
}

// xkey_upsert for a key whose find has just ended at the empty slot idx0
// after nprev occupied slots: the claim is tried there at once (within an
// iteration no other lane inserts this key and nothing is deleted, so the
// slots before it hold other keys); if another key took idx0 meanwhile, the
// walk continues from there as in xkey_upsert.
__device__ inline int64_t xkey_upsert_at(XKey* __restrict__ K, uint64_t mask, uint64_t a, uint64_t b, uint64_t idx0,
                                         int nprev, int* inserted, int* probes, int* err) {
  uint64_t idx = idx0;
  *inserted = 0;
  for (int n = nprev; n < kMaxProbe; ++n) {
    uint64_t ka = n == nprev ? kEmpty : ld_co(&K[idx].ka);
    if (ka == kEmpty) {
      const uint64_t old = atomicCAS((unsigned long long*)&K[idx].ka, (unsigned long long)kEmpty,
                                     (unsigned long long)a);
      if (old == kEmpty) {
        st_co(&K[idx].kb, b);
        *inserted = 1;
        *probes = n + 1;
        return (int64_t)idx;
      }
      ka = old;
    }
    if (ka == a) {
      uint64_t kb = ld_co(&K[idx].kb);
      int spin = 0;
      while (kb == kPending && ++spin < (1 << 20)) kb = ld_co(&K[idx].kb);
      if (kb == kPending) {
        *err |= kErrPublish;
        return -1;
      }
      if (kb == b) {
        *probes = n + 1;
        return (int64_t)idx;
      }
    }
    idx = (idx + 1) & mask;
  }
  *probes = kMaxProbe;
  *err |= kErrTableFull;
  return -1;
}

// ---------------------------------------------------------------- small dense algebra

// Ascending generalised eigenvalues of the pencil (Q, S), n <= kXMax, by one
// thread: Cholesky S = L L^T, M = L^-1 Q L^-T, cyclic Jacobi on M.
__device__ __noinline__ void pencil_eigenvalues(const double* Q, const double* S, int n, double* E) {
  double L[kXMax * kXMax], M[kXMax * kXMax];
  for (int i = 0; i < n * n; ++i) L[i] = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = S[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    const double ljj = sqrt(fmax(s, 1e-300));
    L[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = S[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / ljj;
    }
  }
  // W = L^-1 Q (forward substitution per column), then M = W L^-T
  double W[kXMax * kXMax];
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double t = Q[i * n + c];
      for (int k = 0; k < i; ++k) t -= L[i * n + k] * W[k * n + c];
      W[i * n + c] = t / L[i * n + i];
    }
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double t = W[r * n + i];
      for (int k = 0; k < i; ++k) t -= L[i * n + k] * M[r * n + k];
      M[r * n + i] = t / L[i * n + i];
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double a = 0.5 * (M[i * n + j] + M[j * n + i]);
      M[i * n + j] = M[j * n + i] = a;
    }
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += M[i * n + j] * M[i * n + j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = M[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (M[q * n + q] - M[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double mkp = M[k * n + p], mkq = M[k * n + q];
          M[k * n + p] = c * mkp - s * mkq;
          M[k * n + q] = s * mkp + c * mkq;
        }
        for (int k = 0; k < n; ++k) {
          const double mpk = M[p * n + k], mqk = M[q * n + k];
          M[p * n + k] = c * mpk - s * mqk;
          M[q * n + k] = s * mpk + c * mqk;
        }
      }
  }
  for (int i = 0; i < n; ++i) E[i] = M[i * n + i];
  for (int i = 1; i < n; ++i) {  // insertion sort
    const double v = E[i];
    int j = i - 1;
    while (j >= 0 && E[j] > v) {
      E[j + 1] = E[j];
      --j;
    }
    E[j + 1] = v;
  }
}

// ---------------------------------------------------------------- the step

// argmax candidate: largest |G_j|_inf, ties to the smaller (beta, alpha) key
struct XCand {
  double g;
  uint64_t a, b;
  int64_t slot;
};

__device__ __forceinline__ bool xbetter(const XCand& x, const XCand& y) {
  if (x.g != y.g) return x.g > y.g;
  return key_less(x.a, x.b, y.a, y.b);
}

// workgroup argmax of XCand (a strict total order, so the result does not
// depend on the reduction order); every thread gets the winner
__device__ XCand xblock_argmax(XCand c, XCand* s_c) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    XCand o;
    o.g = __shfl_xor(c.g, off);
    o.a = __shfl_xor(c.a, off);
    o.b = __shfl_xor(c.b, off);
    o.slot = __shfl_xor(c.slot, off);
    if (xbetter(o, c)) c = o;
  }
  if (lane == 0) s_c[w] = c;
  __syncthreads();
  XCand r = s_c[0];
  for (int i = 1; i < nw; ++i)
    if (xbetter(s_c[i], r)) r = s_c[i];
  __syncthreads();
  return r;
}

// workgroup sums of v[0..NS) in a fixed order; every thread gets them
template <int NS>
__device__ void xblock_sums(double (&v)[NS], double* s_red /* kMaxWaves * NS */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double x = v[k];
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(x, off);
      x = (lane & off) ? (o + x) : (x + o);
    }
    if (lane == 0) s_red[w * NS + k] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += s_red[q * NS + k];
    v[k] = t;
  }
  __syncthreads();
}

// The iteration kernel; NS = n states.  One cooperative launch runs up to
// A.nsteps iterations with one device-wide barrier each.  S and Q live in
// every workgroup's shared memory (each keeps an identical copy), the chosen
// row's C and B in registers.  Per iteration:
//   A  every workgroup: lists and H_ii of row i, g, the line search, S and Q
//      updated; workgroup 0 stores C_i' = C_i + eta g;
//   B  each lane one column entry: probe, insert under the compression rule,
//      the row read coherently, B_j += eta H_ji g applied atomically, the
//      candidate |G_j|_inf and H_ji C_j for the recalculation of B_i;
//   -- device-wide barrier --
//   C  every workgroup: combine the partials, B_i = H_ii C_i' + sum H_ji C_j
//      (workgroup 0 adds the correction to the stored B_i atomically, so it
//      commutes with the next iteration's updates of that entry, which use the
//      known values of the previous row instead of reading it), and the next
//      row: i itself or the best candidate, whose row is read after the
//      barrier.
template <int NS, int KIND>  // KIND 0: integrals, 1: momentum-space Hubbard
__global__ void __launch_bounds__(256) k_xiter(XArgs A) {
  constexpr int NN = NS * NS;
  __shared__ Lists L;
  __shared__ double s_red[kMaxWaves * NS];
  __shared__ XCand s_c[kMaxWaves];
  __shared__ double s_Shi[NN], s_Slo[NN], s_Qhi[NN], s_Qlo[NN];
  __shared__ double s_S[NN];  // S before the step, then after it
  __shared__ double s_v[3 * NS];  // C_i, B_i, g
  __shared__ unsigned long long s_ins, s_tot;
  __shared__ int s_err, s_fl, s_probe;
  XCtl* X = A.x;
  if (X->error || X->stopped) return;  // the same in every workgroup
  const Ham H = A.H;
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  const int64_t step0 = X->steps;
  const double shift = X->shift;
  uint64_t ia = X->ia, ib = X->ib;
  int64_t islot = X->islot;
  double d = X->d;
  unsigned long long occupied = X->occupied, inserts = 0;
  double Ci[NS], Bi[NS], pC[NS], pR[NS];
  {
    const double* r = A.R + (size_t)islot * 2 * NS;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      Ci[k] = r[k];
      Bi[k] = r[NS + k];
      pC[k] = pR[k] = 0.0;
    }
  }
  if (tid < NN) {
    s_Shi[tid] = X->S_hi[tid];
    s_Slo[tid] = X->S_lo[tid];
    s_Qhi[tid] = X->Q_hi[tid];
    s_Qlo[tid] = X->Q_lo[tid];
    s_S[tid] = X->S_hi[tid] + X->S_lo[tid];
  }
  uint64_t pa = kEmpty, pb = kEmpty;  // previous row (its B correction may be in flight)
  unsigned target = 0;                // the arrival counter is zeroed before every launch
  int flags = 0, stopped = 0, my_probe = 0;
  int64_t step = 0;
  const int64_t gsz = (int64_t)G * blockDim.x;
  for (; step < A.nsteps; ++step) {
    make_lists_block(ia, ib, KIND ? A.HK.L : H.N, L);
    __syncthreads();  // also: every thread is done with the previous iteration's counters
    if (tid == 0) {
      s_ins = 0;
      s_tot = 0;
      s_err = 0;
      s_fl = 0;
    }
    // ---- A: H_ii of the shifted Hamiltonian, g = 4 B_i + 4 C_i S, the step
    double part = 0.0;
    if (KIND) {
      if (tid < A.HK.L) part = A.HK.eps[tid] * (double)(((ia >> tid) & 1) + ((ib >> tid) & 1));
    } else {
      const int nt = diag_terms(L);
      for (int t = tid; t < nt; t += blockDim.x) part += diag_term(H, L, t);
    }
    double Hii = wg_sum(part, s_red) - shift;
    if (KIND) Hii += A.HK.u * (double)L.na * (double)L.nb;
    double g[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double t = Bi[k];
#pragma unroll
      for (int l = 0; l < NS; ++l) t += Ci[l] * s_S[l * NS + k];
      g[k] = 4.0 * t;
    }
    double gg = 0.0, cg = 0.0, cc = 0.0, gsg = 0.0, ginf = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      gg += g[k] * g[k];
      cg += Ci[k] * g[k];
      cc += Ci[k] * Ci[k];
      ginf = fmax(ginf, fabs(g[k]));
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < NS; ++l) t += s_S[k * NS + l] * g[l];
      gsg += g[k] * t;
    }
    const double w1 = gg, w2 = 2.0 * Hii * gg + 2.0 * cg * cg + 2.0 * cc * gg + 2.0 * gsg;
    const double w3 = 4.0 * gg * cg, w4 = gg * gg;
    const double eta = w4 > 0.0 ? line_search(w1 / w4, w2 / w4, w3 / w4) : 0.0;
    double Cn[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) Cn[k] = Ci[k] + eta * g[k];
    if (tid == 0) {
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        s_v[k] = Ci[k];
        s_v[NS + k] = Bi[k];
        s_v[2 * NS + k] = g[k];
      }
    }
    __syncthreads();  // every thread has read the old S; s_v is complete
    // S' and Q' from the pre-step rows, one element per thread
    if (tid < NN) {
      const int k = tid / NS, l = tid % NS;
      const double Cik = s_v[k], Cil = s_v[l], Bik = s_v[NS + k], Bil = s_v[NS + l];
      const double gk = s_v[2 * NS + k], gl = s_v[2 * NS + l];
      const dd e2 = two_prod(eta, eta);
      const dd gkl = two_prod(gk, gl);
      dd S = dd_add(dd{s_Shi[tid], s_Slo[tid]}, dd_mul_d(dd_add(two_prod(Cik, gl), two_prod(gk, Cil)), eta));
      S = dd_add(S, dd_mul(e2, gkl));
      dd Q = dd_add(dd{s_Qhi[tid], s_Qlo[tid]}, dd_mul_d(dd_add(two_prod(Bik, gl), two_prod(gk, Bil)), eta));
      Q = dd_add(Q, dd_mul_d(dd_mul(e2, gkl), Hii));
      s_Shi[tid] = S.hi;
      s_Slo[tid] = S.lo;
      s_Qhi[tid] = Q.hi;
      s_Qlo[tid] = Q.lo;
      s_S[tid] = dd_val(S);
    }
    if (blockIdx.x == 0 && tid == 0) {
      double* r = A.R + (size_t)islot * 2 * NS;
#pragma unroll
      for (int k = 0; k < NS; ++k) st_co(&r[k], Cn[k]);
    }
    __syncthreads();
    // ---- B: scatter eta H_ji g over the column; candidates; recalculation parts
    XCand best{-1.0, kEmpty, kEmpty, -1};
    double rec[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) rec[k] = 0.0;
    int err = 0;
    unsigned my_ins = 0;
    for (int64_t e = 1 + (int64_t)blockIdx.x * blockDim.x + tid; e < A.n_col; e += gsz) {
      uint64_t ja, jb;
      const double Hj =
          KIND ? column_entry_k(A.HK, L, ia, ib, e, &ja, &jb) : column_entry(H, L, ia, ib, e, 0.0, &ja, &jb);
      if (Hj == 0.0) continue;
      int probes = 0;
      int64_t slot = xkey_find(A.K, A.mask, ja, jb, &probes);
      const bool big = fabs(eta * Hj) * ginf >= A.tau;
      if (slot < 0 && big) {
        // the find ended at an empty slot unless it ran out of probes: the
        // insert starts there
        int ins = 0;
        slot = probes < kMaxProbe
                   ? xkey_upsert_at(A.K, A.mask, ja, jb, (hash_key(ja, jb) + (uint64_t)(probes - 1)) & A.mask,
                                    probes - 1, &ins, &probes, &err)
                   : xkey_upsert(A.K, A.mask, ja, jb, &ins, &probes, &err);
        my_ins += ins;
      }
      my_probe = max(my_probe, probes);
      if (slot < 0) continue;
      double* r = A.R + (size_t)slot * 2 * NS;
      double cj[NS], bj[NS];
      const bool prev = ja == pa && jb == pb;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        cj[k] = prev ? pC[k] : ld_co(&r[k]);
        bj[k] = prev ? pR[k] : ld_co(&r[NS + k]);
      }
      bool anyc = false;
#pragma unroll
      for (int k = 0; k < NS; ++k) anyc = anyc || cj[k] != 0.0;
      if (anyc || big) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const double delta = (eta * Hj) * g[k];
          atomic_add_f64(&r[NS + k], delta);
          bj[k] += delta;
        }
      }
      double gmax = 0.0;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        rec[k] += Hj * cj[k];
        double t = bj[k];
#pragma unroll
        for (int l = 0; l < NS; ++l) t += cj[l] * s_S[l * NS + k];
        gmax = fmax(gmax, fabs(4.0 * t));
      }
      const XCand cnd{gmax, ja, jb, slot};
      if (xbetter(cnd, best)) best = cnd;
    }
    if (my_ins) atomicAdd(&s_ins, (unsigned long long)my_ins);
    if (err) atomicOr(&s_err, err);
    const XCand wb = xblock_argmax(best, s_c);
    xblock_sums<NS>(rec, s_red);
    XPartial* P = A.parts + (size_t)(step & 1) * G;  // double-buffered by parity
    if (tid == 0) {
      XPartial* Q = P + blockIdx.x;
      st_co(&Q->gmax, wb.g);
      st_co(&Q->ka, wb.a);
      st_co(&Q->kb, wb.b);
      st_co(&Q->slot, wb.slot);
#pragma unroll
      for (int k = 0; k < NS; ++k) st_co(&Q->rec[k], rec[k]);
      st_co(&Q->inserts, (int64_t)s_ins);
      st_co(&Q->err, (int64_t)s_err);
    }
    target += G;
    if (!grid_barrier(&X->arrive, target)) flags |= kErrBarrier;
    // ---- C: combine (every workgroup, the same order)
    XCand wc{-1.0, kEmpty, kEmpty, -1};
    double rsum[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) rsum[k] = 0.0;
    unsigned long long ins_tot = 0;
    int fl = 0;
    for (int q = tid; q < G; q += blockDim.x) {  // fixed order per thread
      const XPartial* Q = P + q;
      const XCand c{ld_co(&Q->gmax), ld_co(&Q->ka), ld_co(&Q->kb), ld_co(&Q->slot)};
      if (xbetter(c, wc)) wc = c;
#pragma unroll
      for (int k = 0; k < NS; ++k) rsum[k] += ld_co(&Q->rec[k]);
      ins_tot += (unsigned long long)ld_co(&Q->inserts);
      fl |= (int)ld_co(&Q->err);
    }
    if (ins_tot) atomicAdd(&s_tot, ins_tot);
    if (fl) atomicOr(&s_fl, fl);
    const XCand win = xblock_argmax(wc, s_c);  // its barriers also complete s_tot, s_fl
    xblock_sums<NS>(rsum, s_red);
    flags |= s_fl;
    occupied += s_tot;
    inserts += s_tot;
    if (occupied > A.max_entries) flags |= kErrTableFull;
    // B_i = H_ii C_i' + sum_{j != i} H_ji C_j; the next row
    double Rn[NS];
    double gi = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) Rn[k] = Hii * Cn[k] + rsum[k];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double t = Rn[k];
#pragma unroll
      for (int l = 0; l < NS; ++l) t += Cn[l] * s_S[l * NS + k];
      gi = fmax(gi, fabs(4.0 * t));
    }
    const XCand self{gi, ia, ib, islot};
    const XCand nxt = xbetter(self, win) ? self : win;
    if (blockIdx.x == 0 && tid == 0) {
      double* r = A.R + (size_t)islot * 2 * NS;
#pragma unroll
      for (int k = 0; k < NS; ++k) atomic_add_f64(&r[NS + k], Rn[k] - Bi[k]);
      if (A.tr_SQ) {
        double* t = A.tr_SQ + step * 2 * NN;
        for (int k = 0; k < NN; ++k) {
          t[k] = s_Shi[k] + s_Slo[k];
          t[NN + k] = s_Qhi[k] + s_Qlo[k];
        }
      }
      if (A.tr_a) A.tr_a[step] = ia;
      if (A.tr_b) A.tr_b[step] = ib;
    }
    const double step_norm = fabs(eta) * sqrt(gg);
    d = (step0 + step == 0) ? step_norm : A.theta * d + (1.0 - A.theta) * step_norm;
    pa = ia;
    pb = ib;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      pC[k] = Cn[k];
      pR[k] = Rn[k];
    }
    if (nxt.slot == islot) {
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        Ci[k] = Cn[k];
        Bi[k] = Rn[k];
      }
    } else {  // updated by its owner before the barrier
      const double* r = A.R + (size_t)nxt.slot * 2 * NS;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        Ci[k] = ld_co(&r[k]);
        Bi[k] = ld_co(&r[NS + k]);
      }
    }
    ia = nxt.a;
    ib = nxt.b;
    islot = nxt.slot;
    if (flags) {
      ++step;
      break;
    }
    if (d < A.dx_tol) {
      stopped = 1;
      ++step;
      break;
    }
  }
  // statistics and state write-back
  if (tid == 0) s_probe = 0;
  __syncthreads();
  if (my_probe) atomicMax(&s_probe, my_probe);
  __syncthreads();
  if (tid == 0 && s_probe) atomicMax(&X->max_probe, s_probe);
  if (blockIdx.x == 0) {
    if (tid < NN) {
      X->S_hi[tid] = s_Shi[tid];
      X->S_lo[tid] = s_Slo[tid];
      X->Q_hi[tid] = s_Qhi[tid];
      X->Q_lo[tid] = s_Qlo[tid];
    }
    if (tid == 0) {
      if (flags) atomicOr(&X->error, flags);
      X->d = d;
      X->occupied = occupied;
      X->inserts += inserts;
      X->ia = ia;
      X->ib = ib;
      X->islot = islot;
      X->steps_this_call = step;
      X->stopped = stopped;
    }
  }
}

// ---------------------------------------------------------------- start

struct XInitTask {
  uint64_t a, b;
};

// Start (Sec. 4.1.3, excited-state solver): D_1 = the reference determinant,
// D_2 .. D_n the determinants of lowest H_jj among those connected to it
// (H_j,D1 != 0), equal H_jj ordered by the smaller (beta, alpha) key;
// C^(0) = the unit columns at D_1 .. D_n.

// H_jj of every connected column entry (+inf for zeros and for D_1 itself)
__global__ void __launch_bounds__(256) k_xconn_diag(Ham H, uint64_t a0, uint64_t b0, int64_t n_col,
                                                    double* diag, uint64_t* ka, uint64_t* kb) {
  __shared__ Lists L;
  make_lists_block(a0, b0, H.N, L);
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_col) return;
  uint64_t ja = 0, jb = 0;
  double d = __builtin_huge_val();
  if (e > 0) {
    const double v = column_entry(H, L, a0, b0, e, 0.0, &ja, &jb);
    if (v != 0.0) {
      Lists Lj;
      make_lists_serial(ja, jb, H.N, Lj);
      d = diag_serial(H, Lj);
    }
  }
  diag[e] = d;
  ka[e] = ja;
  kb[e] = jb;
}

// rank of each connected entry by (H_jj, key); ranks below n - 1 become
// D_2 .. D_n (task[1 + rank]); *found counts them
__global__ void __launch_bounds__(256) k_xconn_rank(const double* diag, const uint64_t* ka, const uint64_t* kb,
                                                    int64_t n_col, int n, XInitTask* task, int* found) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_col) return;
  const double v = diag[e];
  if (v == __builtin_huge_val()) return;
  int rank = 0;
  for (int64_t f = 1; f < n_col && rank < n - 1; ++f) {
    const double w = diag[f];
    if (w < v || (w == v && f != e && key_less(ka[f], kb[f], ka[e], kb[e]))) ++rank;
  }
  if (rank < n - 1) {
    task[1 + rank] = XInitTask{ka[e], kb[e]};
    atomicAdd(found, 1);
  }
}

// store the start rows C^(0)
__global__ void k_xinit_insert(XKey* K, double* R, uint64_t mask, const XInitTask* task, const double* coef,
                               int m, int n, XCtl* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int ins = 0, probes = 0, err = 0;
  const int64_t s = xkey_upsert(K, mask, task[i].a, task[i].b, &ins, &probes, &err);
  if (s < 0) {
    atomicOr(&x->error, err ? err : kErrTableFull);
    return;
  }
  for (int k = 0; k < n; ++k) R[(size_t)s * 2 * n + k] = coef[i * n + k];
  if (ins) {
    atomicAdd(&x->occupied, 1ull);
    atomicAdd(&x->inserts, 1ull);
  }
}

// B^(0) = H C^(0): grid (column chunks, m start determinants)
__global__ void __launch_bounds__(256) k_xinit_scatter(Ham H, XKey* K, double* R, uint64_t mask,
                                                       const XInitTask* task, const double* coef, int n,
                                                       int64_t n_col, double shift, XCtl* x) {
  __shared__ Lists L;
  __shared__ double s_diag;
  const XInitTask t = task[blockIdx.y];
  if (threadIdx.x == 0) {
    make_lists_serial(t.a, t.b, H.N, L);
    s_diag = diag_serial(H, L) - shift;
  }
  __syncthreads();
  unsigned long long ins_cnt = 0;
  int err = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_col;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t ja, jb;
    const double Hj = column_entry(H, L, t.a, t.b, e, s_diag, &ja, &jb);
    if (Hj == 0.0) continue;
    int ins = 0, probes = 0;
    const int64_t s = xkey_upsert(K, mask, ja, jb, &ins, &probes, &err);
    if (s < 0) break;
    for (int k = 0; k < n; ++k) atomic_add_f64(&R[(size_t)s * 2 * n + n + k], Hj * coef[blockIdx.y * n + k]);
    ins_cnt += ins;
  }
  if (err) atomicOr(&x->error, err);
  if (ins_cnt) {
    atomicAdd(&x->occupied, ins_cnt);
    atomicAdd(&x->inserts, ins_cnt);
  }
}

// B^(0) = (H - shift) C^(0) for the momentum-space model: grid (column
// chunks, m start determinants)
__global__ void __launch_bounds__(256) k_xinit_scatter_k(HamK HK, XKey* K, double* R, uint64_t mask,
                                                         const XInitTask* task, const double* coef, int n,
                                                         int na, int nb, double shift, XCtl* x) {
  __shared__ Lists L;
  __shared__ double s_diag;
  const XInitTask t = task[blockIdx.y];
  if (threadIdx.x == 0) {
    make_lists_serial(t.a, t.b, HK.L, L);
    double d = HK.u * (double)na * (double)nb - shift;
    for (int i = 0; i < L.na; ++i) d += HK.eps[L.oa[i]];
    for (int i = 0; i < L.nb; ++i) d += HK.eps[L.ob[i]];
    s_diag = d;
  }
  __syncthreads();
  const int64_t n_col = column_count_k(HK.L, na, nb);
  unsigned long long ins_cnt = 0;
  int err = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_col;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t ja = t.a, jb = t.b;
    const double Hj = e == 0 ? s_diag : column_entry_k(HK, L, t.a, t.b, e, &ja, &jb);
    if (Hj == 0.0) continue;
    int ins = 0, probes = 0;
    const int64_t s = xkey_upsert(K, mask, ja, jb, &ins, &probes, &err);
    if (s < 0) break;
    for (int k = 0; k < n; ++k) atomic_add_f64(&R[(size_t)s * 2 * n + n + k], Hj * coef[blockIdx.y * n + k]);
    ins_cnt += ins;
  }
  if (err) atomicOr(&x->error, err);
  if (ins_cnt) {
    atomicAdd(&x->occupied, ins_cnt);
    atomicAdd(&x->inserts, ins_cnt);
  }
}

// S = C^T C and Q = C^T B over the start rows (double-double, one thread)
__global__ void k_xinit_matrices(const XKey* K, const double* R, uint64_t mask, const XInitTask* task, int m,
                                 int n, XCtl* x) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  dd S[kXMax * kXMax], Q[kXMax * kXMax];
  for (int k = 0; k < n * n; ++k) S[k] = Q[k] = dd{0.0, 0.0};
  for (int i = 0; i < m; ++i) {
    int probes;
    const int64_t s = xkey_find(K, mask, task[i].a, task[i].b, &probes);
    if (s < 0) continue;
    const double* r = R + (size_t)s * 2 * n;
    for (int k = 0; k < n; ++k)
      for (int l = 0; l < n; ++l) {
        S[k * n + l] = dd_add(S[k * n + l], two_prod(r[k], r[l]));
        Q[k * n + l] = dd_add(Q[k * n + l], two_prod(r[k], r[n + l]));
      }
  }
  for (int k = 0; k < n; ++k)  // C^T H C is symmetric: average the two halves
    for (int l = k + 1; l < n; ++l) {
      const dd a = dd_add(Q[k * n + l], Q[l * n + k]);
      const dd h{0.5 * a.hi, 0.5 * a.lo};
      Q[k * n + l] = Q[l * n + k] = h;
    }
  for (int k = 0; k < n * n; ++k) {
    x->S_hi[k] = S[k].hi;
    x->S_lo[k] = S[k].lo;
    x->Q_hi[k] = Q[k].hi;
    x->Q_lo[k] = Q[k].lo;
  }
}

// first coordinate: argmax of |G_j|_inf over every stored entry (one
// workgroup per slice, then one thread over the slices)
__global__ void __launch_bounds__(256) k_xselect_table(const XKey* K, const double* R, uint64_t nslots,
                                                       const XCtl* x, XPartial* parts) {
  __shared__ XCand s_c[kMaxWaves];
  const int n = x->n;
  double S[kXMax * kXMax];
  for (int k = 0; k < n * n; ++k) S[k] = x->S_hi[k] + x->S_lo[k];
  XCand best{-1.0, kEmpty, kEmpty, -1};
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    if (K[s].ka == kEmpty) continue;
    const double* r = R + s * 2 * n;
    double gmax = 0.0;
    for (int k = 0; k < n; ++k) {
      double t = r[n + k];
      for (int l = 0; l < n; ++l) t += r[l] * S[l * n + k];
      gmax = fmax(gmax, fabs(4.0 * t));
    }
    const XCand c{gmax, K[s].ka, K[s].kb, (int64_t)s};
    if (xbetter(c, best)) best = c;
  }
  const XCand w = xblock_argmax(best, s_c);
  if (threadIdx.x == 0) {
    parts[blockIdx.x].gmax = w.g;
    parts[blockIdx.x].ka = w.a;
    parts[blockIdx.x].kb = w.b;
    parts[blockIdx.x].slot = w.slot;
  }
}

__global__ void k_xselect_final(const XPartial* parts, int np, XCtl* x) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  XCand w{-1.0, kEmpty, kEmpty, -1};
  for (int i = 0; i < np; ++i) {
    const XCand c{parts[i].gmax, parts[i].ka, parts[i].kb, parts[i].slot};
    if (xbetter(c, w)) w = c;
  }
  x->ia = w.a;
  x->ib = w.b;
  x->islot = w.slot;
}

// energies of traced steps: one thread per step
__global__ void __launch_bounds__(64) k_xtrace_energies(const double* SQ, int64_t steps, int n, double shift,
                                                         double* E) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= steps) return;
  const double* t = SQ + i * 2 * n * n;
  pencil_eigenvalues(t + n * n, t, n, E + i * n);
  for (int k = 0; k < n; ++k) E[i * n + k] += shift;
}

// energies now: the pencil (Q, S), plus the shift
__global__ void k_xenergies(const XCtl* x, double* E) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = x->n;
  double S[kXMax * kXMax], Q[kXMax * kXMax];
  for (int k = 0; k < n * n; ++k) {
    S[k] = x->S_hi[k] + x->S_lo[k];
    Q[k] = x->Q_hi[k] + x->Q_lo[k];
  }
  pencil_eigenvalues(Q, S, n, E);
  for (int k = 0; k < n; ++k) E[k] += x->shift;
}

// rows of every stored determinant (compaction by one atomic per entry)
__global__ void __launch_bounds__(256) k_xexport(const XKey* K, const double* R, uint64_t nslots, int n,
                                                 uint64_t* ka, uint64_t* kb, double* C, double* B, int64_t cap,
                                                 unsigned long long* count) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    if (K[s].ka == kEmpty) continue;
    const unsigned long long q = atomicAdd(count, 1ull);
    if ((int64_t)q >= cap) continue;
    ka[q] = K[s].ka;
    kb[q] = K[s].kb;
    for (int k = 0; k < n; ++k) {
      C[q * n + k] = R[s * 2 * n + k];
      B[q * n + k] = R[s * 2 * n + n + k];
    }
  }
}

__global__ void k_xclear(XKey* K, double* R, uint64_t nslots, int n) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    K[s].ka = kEmpty;
    K[s].kb = kPending;
    for (int k = 0; k < 2 * n; ++k) R[s * 2 * n + k] = 0.0;
  }
}
