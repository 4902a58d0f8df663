// Orbital optimisation around FCI, OptOrbFCI (paper Sec. 3.4, eq. (subopt),
// Algorithm 4), device side.  Included into cdfci.hip inside its kernel
// namespace.
//
// The N orbitals of the FCI space are the columns of U (M x N).  The
// integrals in them are h' = U^T h U and the four-index transform of
// (pq|rs); with the RDMs of the FCI ground state held fixed,
//   P4(U) = sum h'_pq gamma_pq + 1/2 sum (pq|rs)' Gamma_pqrs
// and, with Gamma symmetrised over the eight index permutations that leave
// (pq|rs) unchanged (P4 sees only that part), its gradient in U is
//   h U (gamma + gamma^T) + 2 sum_jkl W_ajkl Gs_ijkl,
//   W_ajkl = sum_qrs (aq|rs) U_qj U_rk U_sl,
// the four positions of U in the two-body term giving equal shares.

// Contraction of one index of a 4-index tensor with U: out has the sizes of
// in except size N at position pos, out[..i..] = sum_a in[..a..] U[a][i]
// (a < M).  Row-major, one thread per output element.
__global__ void __launch_bounds__(256) k_orb_contract(const double* __restrict__ in, double* __restrict__ out,
                                                      const double* __restrict__ U, int M, int N, int d0, int d1,
                                                      int d2, int d3, int pos) {
  int dims[4] = {d0, d1, d2, d3};
  dims[pos] = N;
  const int64_t total = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= total) return;
  int idx[4];
  int64_t r = o;
  for (int q = 3; q >= 0; --q) {
    idx[q] = (int)(r % dims[q]);
    r /= dims[q];
  }
  const int in_dims[4] = {d0, d1, d2, d3};
  int64_t stride = 1;
  for (int q = 3; q > pos; --q) stride *= in_dims[q];
  int64_t base = 0;
  for (int q = 0; q < 4; ++q) base = base * in_dims[q] + (q == pos ? 0 : idx[q]);
  const int i = idx[pos];
  double s = 0.0;
  for (int a = 0; a < M; ++a) s += in[base + a * stride] * U[(int64_t)a * N + i];
  out[o] = s;
}

// part[block] = sum over the block's share of x_k y_k (fixed order per
// thread, then the workgroup sum); the host adds the parts in order
__global__ void __launch_bounds__(256) k_orb_dot(const double* __restrict__ x, const double* __restrict__ y,
                                                 int64_t n, double* part) {
  __shared__ double s_red[4];
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    s += x[k] * y[k];
  s = wg_sum(s, s_red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// grad2[a][i] = 2 sum_jkl W[a][jkl] Gs[i][jkl]; one workgroup per (a, i)
__global__ void __launch_bounds__(256) k_orb_grad2(const double* __restrict__ W, const double* __restrict__ Gs,
                                                   int M, int N, double* grad2) {
  __shared__ double s_red[4];
  const int a = blockIdx.x / N, i = blockIdx.x % N;
  const int64_t n3 = (int64_t)N * N * N;
  const double* w = W + (int64_t)a * n3;
  const double* g = Gs + (int64_t)i * n3;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n3; k += blockDim.x) s += w[k] * g[k];
  s = wg_sum(s, s_red);
  if (threadIdx.x == 0) grad2[(int64_t)a * N + i] = 2.0 * s;
}
