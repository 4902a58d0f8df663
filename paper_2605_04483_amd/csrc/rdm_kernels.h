// Reverse pass of E(h, eri) = c^T H c / c^T c with c held fixed: the
// spin-summed reduced density matrices of the truncated, normalised
// wavefunction and the orbital-rotation gradient (Sec. 3.4, eq. (subopt) at
// U = I).  Included into cdfci.hip inside its kernel namespace after
// mcd_kernels.h.
//
//   gamma_pq   = sum_s <a+_ps a_qs>                      1-RDM
//   Gamma_pqrs = sum_st <a+_ps a+_rt a_st a_qs>          2-RDM, chemist order
//   E          = sum h gamma + 1/2 sum (pq|rs) Gamma
//   kappa_pq   = 2 (F_pq - F_qp),  F = h gamma + ERI_(p,rst) Gamma_(q,rst)^T
//
// Off-diagonal part.  Every unordered pair of support determinants (J, I)
// connected by an excitation is visited once, from the column of the smaller
// key J.  With I = s a+_r a_p J (single, spin t) and w = s c_I c_J the
// nonzero elements of <I|op|J> are gamma_rp = w and, for every other occupied
// spin-orbital k of J,  Gamma_rpkk = Gamma_kkrp = w  and, when k has spin t,
// Gamma_rkkp = Gamma_kprk = -w.  With I = s a+_r a+_s a_q a_p J (double):
// Gamma_rpsq = Gamma_sqrp = w and, for equal spins, Gamma_rqsp = Gamma_sprq = -w.
// The elements come in particle-swap pairs (Gamma_abcd, Gamma_cdab) and
// <J|op|I> is their Hermitian image (gamma_ab -> gamma_ba, Gamma_abcd ->
// Gamma_badc), so only one member of each swap pair is accumulated (Z) and
//   Gamma_pqrs = Z_pqrs + Z_rspq + Z_qpsr + Z_srqp,  gamma_pq = Y_pq + Y_qp
// restores the rest (where two images fall on one element, the sum counts it
// twice, as the direct rule does).
// Diagonal part (I = J, weight c_J^2): gamma_pp per occupied spin-orbital,
// Gamma_pprr per ordered pair of distinct occupied spin-orbitals and
// -Gamma_prrp per ordered pair of equal spin; added after symmetrisation.

__device__ __forceinline__ size_t g4(int N, int p, int q, int r, int s) {
  return (((size_t)p * N + q) * N + r) * N + s;
}

// every stored entry with c != 0, as a dense candidate list
__global__ void __launch_bounds__(256) k_rdm_nonzero(const Slot* T, uint64_t nslots, unsigned* cand,
                                                     McState* st, uint64_t cap) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const Slot s = T[i];
    if (s.ka == kEmpty || s.c == 0.0) continue;
    unsigned long long k = atomicAdd(&st->n_dense, 1ull);
    if (k < cap) cand[k] = (unsigned)i;
  }
}

// partial sums of c^2 over the chosen support, one per workgroup
__global__ void __launch_bounds__(256) k_rdm_norm(const Slot* T, const int64_t* sel_slot, int64_t n,
                                                  double* part) {
  __shared__ double s_red[4];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double c = T[sel_slot[i]].c;
    v += c * c;
  }
  const double t = wg_sum(v, s_red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// support table: the chosen determinants with c / ||c||, plus dense copies
__global__ void __launch_bounds__(256) k_rdm_build(const Slot* T, const int64_t* sel_slot, int64_t n,
                                                   const double* norm2, Slot* S, uint64_t smask,
                                                   uint64_t* sup_a, uint64_t* sup_b, double* sup_c,
                                                   int* err) {
  const double inv = 1.0 / sqrt(*norm2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Slot t = T[sel_slot[i]];
    int ins = 0, probes = 0, e = 0;
    SlotVal v;
    const int64_t s = table_upsert(S, smask, t.ka, t.kb, &ins, &probes, &e, &v);
    if (s < 0) {
      atomicOr(err, kErrTableFull);
      continue;
    }
    const double c = t.c * inv;
    S[s].c = c;
    sup_a[i] = t.ka;
    sup_b[i] = t.kb;
    sup_c[i] = c;
  }
}

// lookup in the finished (read-only) support table: plain cached loads
__device__ __forceinline__ bool support_find(const Slot* __restrict__ S, uint64_t mask, uint64_t a,
                                             uint64_t b, double* c) {
  uint64_t idx = hash_key(a, b) & mask;
  for (int n = 0; n < kMaxProbe; ++n) {
    const Slot v = S[idx];
    if (v.ka == kEmpty) return false;
    if (v.ka == a && v.kb == b) {
      *c = v.c;
      return true;
    }
    idx = (idx + 1) & mask;
  }
  return false;
}

// off-diagonal pairs: workgroups stride over the support determinants J and
// sweep each column with one entry per thread
__global__ void __launch_bounds__(256) k_rdm_pairs(Ham H, const Slot* __restrict__ S, uint64_t smask,
                                                   const uint64_t* sup_a, const uint64_t* sup_b,
                                                   const double* sup_c, int64_t n, int64_t n_col,
                                                   double* Y1, double* Z, double* e_acc) {
  __shared__ Lists L;
  __shared__ double s_red[4];
  const int N = H.N;
  double ehc = 0.0;
  for (int64_t d = blockIdx.x; d < n; d += gridDim.x) {
    const uint64_t a = sup_a[d], b = sup_b[d];
    const double cj = sup_c[d];
    __syncthreads();
    make_lists_block(a, b, N, L);
    __syncthreads();
    for (int64_t e = 1 + threadIdx.x; e < n_col; e += blockDim.x) {
      uint64_t ia, ib;
      const Excitation x = decode_excitation(L, a, b, (uint32_t)e, &ia, &ib);
      if (!key_less(a, b, ia, ib)) continue;  // each unordered pair once
      double ci;
      if (!support_find(S, smask, ia, ib, &ci)) continue;
      const double w = x.neg ? -ci * cj : ci * cj;
      const int p = x.p, q = x.q, r = x.r, s = x.s;
      if (x.type <= 2) {
        const bool al = x.type == 1;
        atomic_add_f64(&Y1[r * N + p], w);
        const int8_t* same = al ? L.oa : L.ob;
        const int8_t* other = al ? L.ob : L.oa;
        const int ns = al ? L.na : L.nb, no = al ? L.nb : L.na;
        for (int t = 0; t < ns; ++t) {
          const int k = same[t];
          if (k == p) continue;
          atomic_add_f64(&Z[g4(N, r, p, k, k)], w);
          atomic_add_f64(&Z[g4(N, r, k, k, p)], -w);
        }
        for (int t = 0; t < no; ++t) {
          const int k = other[t];
          atomic_add_f64(&Z[g4(N, r, p, k, k)], w);
        }
        const double hv = al ? single_value(H, p, r, L.oa, L.na, L.ob, L.nb)
                             : single_value(H, p, r, L.ob, L.nb, L.oa, L.na);
        ehc += 2.0 * w * hv;
      } else {
        atomic_add_f64(&Z[g4(N, r, p, s, q)], w);
        double v = ERI(H, r, p, s, q);
        if (x.type != 5) {
          atomic_add_f64(&Z[g4(N, r, q, s, p)], -w);
          v -= ERI(H, r, q, s, p);
        }
        ehc += 2.0 * w * v;
      }
    }
  }
  const double t = wg_sum(ehc, s_red);
  if (threadIdx.x == 0 && t != 0.0) atomic_add_f64(e_acc, t);
}

// gamma = Y + Y^T;  Gamma_pqrs = Z_pqrs + Z_rspq + Z_qpsr + Z_srqp
__global__ void __launch_bounds__(256) k_rdm_symmetrize(const double* Y1, const double* Z, int N,
                                                        double* g1, double* g2) {
  const size_t N2 = (size_t)N * N, N4 = N2 * N2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N4;
       i += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(i % N), r = (int)((i / N) % N), q = (int)((i / N2) % N), p = (int)(i / (N2 * N));
    g2[i] = Z[i] + Z[g4(N, r, s, p, q)] + Z[g4(N, q, p, s, r)] + Z[g4(N, s, r, q, p)];
    if (i < N2) {
      const int a = (int)(i / N), b = (int)(i % N);
      g1[i] = Y1[i] + Y1[(size_t)b * N + a];
    }
  }
}

// diagonal terms and c_J^2 H_JJ: per-workgroup shared accumulators, flushed
// once.  Shared layout: [N] gamma_pp, [N*N] Gamma_pprr, [N*N] Gamma_prrp.
__global__ void __launch_bounds__(256) k_rdm_diag(Ham H, const uint64_t* sup_a, const uint64_t* sup_b,
                                                  const double* sup_c, int64_t n, double* g1, double* g2,
                                                  double* e_acc) {
  extern __shared__ double sm[];
  __shared__ Lists L;
  __shared__ double s_red[4];
  const int N = H.N;
  double* d1 = sm;
  double* d2 = sm + N;
  double* d3 = sm + N + N * N;
  for (int i = threadIdx.x; i < N + 2 * N * N; i += blockDim.x) sm[i] = 0.0;
  double ehc = 0.0;
  for (int64_t d = blockIdx.x; d < n; d += gridDim.x) {
    __syncthreads();
    make_lists_block(sup_a[d], sup_b[d], N, L);
    __syncthreads();
    const double w = sup_c[d] * sup_c[d];
    const int na = L.na, nt = L.na + L.nb;
    for (int P = threadIdx.x; P < nt; P += blockDim.x) {
      const int p = P < na ? L.oa[P] : L.ob[P - na];
      atomicAdd(&d1[p], w);
    }
    for (int t = threadIdx.x; t < nt * nt; t += blockDim.x) {
      const int P = t / nt, R = t % nt;
      if (P == R) continue;
      const int p = P < na ? L.oa[P] : L.ob[P - na];
      const int r = R < na ? L.oa[R] : L.ob[R - na];
      atomicAdd(&d2[p * N + r], w);
      if ((P < na) == (R < na)) atomicAdd(&d3[p * N + r], -w);
    }
    double part = 0.0;
    const int ntm = diag_terms(L);
    for (int t = threadIdx.x; t < ntm; t += blockDim.x) part += diag_term(H, L, t);
    ehc += w * wg_sum(part, s_red);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x)
    if (d1[i] != 0.0) atomic_add_f64(&g1[i * N + i], d1[i]);
  for (int i = threadIdx.x; i < N * N; i += blockDim.x) {
    const int p = i / N, r = i % N;
    if (d2[i] != 0.0) atomic_add_f64(&g2[g4(N, p, p, r, r)], d2[i]);
    if (d3[i] != 0.0) atomic_add_f64(&g2[g4(N, p, r, r, p)], d3[i]);
  }
  if (threadIdx.x == 0) atomic_add_f64(e_acc, ehc);
}

// F2 = ERI_(p, rst) Gamma_(q, rst)^T on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): one wave per 16x16 output tile and K slice,
// partial tiles added atomically.  Operand layout of the instruction: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register v of
// lane l holds D[4 v + l / 16][l % 16] (checked with one-hot operands).
constexpr int kKappaSlice = 2048;

__global__ void __launch_bounds__(64) k_kappa_mfma(const double* __restrict__ eri,
                                                   const double* __restrict__ g2, int N, double* F2) {
  const int tiles = (N + 15) / 16;
  const int tp = blockIdx.x / tiles, tq = blockIdx.x % tiles;
  const int lane = threadIdx.x;
  const int64_t K = (int64_t)N * N * N;
  const int64_t k0 = (int64_t)blockIdx.y * kKappaSlice;
  const int64_t k1 = min(K, k0 + (int64_t)kKappaSlice);
  const int row = lane % 16, kk = lane / 16;
  const int pa = tp * 16 + row, qb = tq * 16 + row;
  const double* ar = eri + (size_t)min(pa, N - 1) * K;
  const double* br = g2 + (size_t)min(qb, N - 1) * K;
  typedef double v4d __attribute__((ext_vector_type(4)));
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k = k0; k < k1; k += 4) {
    const int64_t kc = k + kk;
    const double av = (pa < N && kc < k1) ? ar[kc] : 0.0;
    const double bv = (qb < N && kc < k1) ? br[kc] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  const int col = tq * 16 + lane % 16;
  for (int v = 0; v < 4; ++v) {
    const int rr = tp * 16 + 4 * v + lane / 16;
    if (rr < N && col < N) atomic_add_f64(&F2[rr * N + col], acc[v]);
  }
}

// F = h gamma + F2;  kappa = gE 2 (F - F^T);  dh = gE gamma
__global__ void __launch_bounds__(256) k_kappa_finish(const double* h, const double* g1, const double* F2,
                                                      int N, double gE, double* kappa, double* dh) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N * N; i += gridDim.x * blockDim.x) {
    const int p = i / N, q = i % N;
    double f_pq = F2[p * N + q], f_qp = F2[q * N + p];
    for (int r = 0; r < N; ++r) {
      f_pq += h[p * N + r] * g1[r * N + q];
      f_qp += h[q * N + r] * g1[r * N + p];
    }
    kappa[i] = gE * 2.0 * (f_pq - f_qp);
    dh[i] = gE * g1[i];
  }
}

// partial sums of sum h gamma + 1/2 sum eri Gamma, one per workgroup; then
// Gamma is overwritten in place by deri = gE Gamma / 2
__global__ void __launch_bounds__(256) k_rdm_outputs(const double* h, const double* eri, const double* g1,
                                                     double* g2, int N, double gE, double* e_part) {
  __shared__ double s_red[4];
  const size_t N2 = (size_t)N * N, N4 = N2 * N2;
  double e = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N4;
       i += (size_t)gridDim.x * blockDim.x) {
    const double G = g2[i];
    e += 0.5 * eri[i] * G;
    g2[i] = 0.5 * gE * G;
  }
  if (blockIdx.x == 0)
    for (size_t i = threadIdx.x; i < N2; i += blockDim.x) e += h[i] * g1[i];
  const double t = wg_sum(e, s_red);
  if (threadIdx.x == 0) e_part[blockIdx.x] = t;
}
