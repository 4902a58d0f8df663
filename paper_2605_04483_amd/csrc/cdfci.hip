// Coordinate-descent FCI on MI355X: kernels and the C ABI (include/cdfci.h).
//
// Hot path of one single-coordinate iteration (paper Sec. 3.1, Algorithm 1),
// executed by a persistent cooperative kernel with one device-wide barrier
// per iteration:
//   A  every workgroup redundantly: lists of the chosen determinant D, H_DD,
//      exact line search (Appendix A), mu/alpha update in double-double;
//      workgroup 0 stores c_D + eta;
//   B  all lanes over the column of D (singles and doubles, Sec. 4.3): key,
//      Slater-Condon entry, hash probe (insert under the compression rule),
//      FP64 atomic b_j += eta H_jD, gather of c_j for the recalculation of b_D,
//      gradient |4 b_j + 4 mu c_j| of the touched entry and a workgroup
//      argmax (ties: smaller (beta, alpha) key);
//   -- device-wide barrier --
//   C  every workgroup redundantly: combine the per-workgroup argmax and the
//      recalculation sum, giving b_D (Sec. 3.1 eq. (recalculate-b)) and the
//      next coordinate; workgroup 0 applies b_D's correction atomically.
// The next iteration's candidates are exactly the column just scattered plus
// D itself (Alg. 1: argmax over I_H(i)), so selection fuses into the scatter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cdfci.h"
#include "device.h"

using namespace cdfci;

namespace {

thread_local std::string g_last_error;

// Staging memory of cdfci_column_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code uses only the device
// address resolved per device at context set-up.
constexpr int64_t kNoAllocMaxEntries = 1 << 18;  // column entries (keys 16 B + value 8 B each): 6 MiB
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocMaxEntries * (2 * sizeof(uint64_t) + sizeof(double))];
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// resolve this device's address of `scratch` once (the device must be current)
hipError_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch_ptr[device] = p;
  return e;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) {                                                             \
      g_last_error = std::string(#expr) + ": " + hipGetErrorString(_e);                 \
      return CDFCI_ERR_HIP;                                                             \
    }                                                                                   \
  } while (0)

// Control block in device memory: the solver's scalar state between launches.
struct Ctl {
  double mu_hi, mu_lo, al_hi, al_lo;  // mu = c.c, alpha = c.Hc (double-double)
  double d;                           // damped step accumulator
  double energy;
  uint64_t sel_a, sel_b;              // next coordinate to update
  int64_t sel_slot;
  double sel_c, sel_b_val;            // its c and b (b includes every correction)
  int64_t steps;                      // iterations since init
  unsigned long long occupied;        // stored determinants
  unsigned long long inserts;
  unsigned long long probes;          // slots inspected by multicoordinate scatters
  unsigned long long atomics;         // FP64 atomic b updates of multicoordinate scatters
  int error;
  int stopped;
  int max_probe;
  unsigned barrier;                   // device-wide barrier arrival counter
  int64_t steps_this_call;
  // wall-clock ticks spent by workgroup 0 per phase (A, B, barrier wait, C)
  unsigned long long t_phase[4];
};

// Per-workgroup result of phase B (one per workgroup and iteration parity).
struct alignas(64) Partial {
  double g;
  uint64_t a, b;
  int64_t slot;
  double bnew, c;
  double recalc;
  int64_t info;  // inserts << 8 | error bits of the workgroup
};

struct Cand {
  double g;
  uint64_t a, b;
  int64_t slot;
  double bnew, c;
};

__device__ __forceinline__ bool better(const Cand& x, const Cand& y) {
  if (x.g != y.g) return x.g > y.g;
  return key_less(x.a, x.b, y.a, y.b);
}

__device__ __forceinline__ Cand shfl_cand(const Cand& c, int src) {
  Cand o;
  o.g = __shfl(c.g, src);
  o.a = __shfl(c.a, src);
  o.b = __shfl(c.b, src);
  o.slot = __shfl(c.slot, src);
  o.bnew = __shfl(c.bnew, src);
  o.c = __shfl(c.c, src);
  return o;
}

// Deterministic workgroup argmax + sum (identical result in every workgroup for
// identical inputs).  Uses shared scratch of blockDim/64 entries.
template <int MAXW>
__device__ void block_reduce(Cand& best, double& sum, Cand* s_cand, double* s_sum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    Cand o = shfl_cand(best, lane ^ off);
    double so = __shfl_xor(sum, off);
    // `better` is a strict total order on (g, key), so both partners keep the
    // same winner; the sum is formed lower-lane-first on both sides
    const bool take = better(o, best);
    best.g = take ? o.g : best.g;
    best.a = take ? o.a : best.a;
    best.b = take ? o.b : best.b;
    best.slot = take ? o.slot : best.slot;
    best.bnew = take ? o.bnew : best.bnew;
    best.c = take ? o.c : best.c;
    sum = (lane & off) ? (so + sum) : (sum + so);
  }
  if (lane == 0) {
    s_cand[w] = best;
    s_sum[w] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Cand b = s_cand[0];
    double s = s_sum[0];
    for (int i = 1; i < nw; ++i) {
      if (better(s_cand[i], b)) b = s_cand[i];
      s += s_sum[i];
    }
    s_cand[0] = b;
    s_sum[0] = s;
  }
  __syncthreads();
  best = s_cand[0];
  sum = s_sum[0];
  __syncthreads();
}

// Device-wide barrier with a spin bound; returns false on timeout.
// Every access to data shared between workgroups inside the persistent kernel
// is an agent-scope atomic (serviced at the coherence point), so the barrier
// only has to order them: each wave drains its outstanding memory operations
// (s_waitcnt) before the workgroup arrives, and nothing is read before the
// arrival count is seen.  No L2 write-back or invalidate is issued.
__device__ bool grid_barrier(unsigned* counter, unsigned target) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int spins = 0;
    ok = 1;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1 << 27)) {
        ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

__device__ __forceinline__ void partial_store(Partial* p, const Cand& c, double recalc) {
  st_co(&p->g, c.g);
  st_co(&p->a, c.a);
  st_co(&p->b, c.b);
  st_co(&p->slot, c.slot);
  st_co(&p->bnew, c.bnew);
  st_co(&p->c, c.c);
  st_co(&p->recalc, recalc);
}
__device__ __forceinline__ Cand partial_load(const Partial* p, double* recalc) {
  Cand c;
  c.g = ld_co(&p->g);
  c.a = ld_co(&p->a);
  c.b = ld_co(&p->b);
  c.slot = ld_co(&p->slot);
  c.bnew = ld_co(&p->bnew);
  c.c = ld_co(&p->c);
  *recalc = ld_co(&p->recalc);
  return c;
}

constexpr int kMaxWaves = 4;  // workgroups of at most 256 threads

// ---------------------------------------------------------------------------
// Persistent single-coordinate kernel.

struct Cd1Args {
  Ham H;
  Slot* T;
  uint64_t mask;
  uint64_t max_entries;
  Ctl* ctl;
  Partial* parts;  // 2 * gridDim.x
  int64_t nsteps;
  int64_t n_col;   // entries per column (diagonal included)
  double tau, theta, dx_tol;
  double* tr_E;
  uint64_t* tr_a;
  uint64_t* tr_b;
  double* tr_eta;
};

__global__ void __launch_bounds__(256) k_cd1(Cd1Args A) {
  __shared__ Lists L;
  __shared__ Cand s_cand[kMaxWaves];
  __shared__ double s_sum[kMaxWaves];
  __shared__ double s_bc[8];
  __shared__ unsigned long long s_info, s_ins_sum;
  __shared__ int s_flags;

  const Ham H = A.H;
  Ctl* ctl = A.ctl;
  const int G = gridDim.x;
  const int tid = threadIdx.x;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + tid;
  const int64_t gsz = (int64_t)G * blockDim.x;

  // scalar state, identical in every workgroup
  dd mu{ctl->mu_hi, ctl->mu_lo}, al{ctl->al_hi, ctl->al_lo};
  double d = ctl->d;
  uint64_t sa = ctl->sel_a, sb = ctl->sel_b;
  int64_t sslot = ctl->sel_slot;
  double sc = ctl->sel_c, sbv = ctl->sel_b_val;
  const int64_t step0 = ctl->steps;
  unsigned long long occupied = ctl->occupied, inserts = 0;
  uint64_t pa = kEmpty, pb = kEmpty;  // previous coordinate (pending correction)
  double pR = 0.0;
  unsigned target = 0;  // the arrival counter is zeroed before every launch
  int64_t step = 0;
  int stopped = 0, flags = 0;
  int my_probe = 0;

  // phase timers of workgroup 0 (wall-clock ticks), compiled in only for
  // profiling builds (-DCDFCI_PHASE_TIMING)
  unsigned long long tp0 = 0, tp1 = 0, tp2 = 0, tp3 = 0;
#ifdef CDFCI_PHASE_TIMING
  unsigned long long t_last = wall_clock64();
#define CDFCI_TICK(acc)                          \
  if (blockIdx.x == 0 && tid == 0) {             \
    unsigned long long t_now = wall_clock64();   \
    acc += t_now - t_last;                       \
    t_last = t_now;                              \
  }
#else
#define CDFCI_TICK(acc)
#endif
  for (; step < A.nsteps; ++step) {
    // ---- phase A: lists of D; every lane forms its first column entry and
    // issues the first probe load of it; while those loads are in flight,
    // wave 0 forms H_DD (its integrals loaded before the entry's, summed by a
    // fixed-order wave sum with no workgroup barrier) and takes the line
    // search; then the probes complete
    make_lists_block(sa, sb, H.N, L);
    __syncthreads();
    const int nt = diag_terms(L);
    DiagLoad dg0{0.0, 0.0, 0.0}, dg1{0.0, 0.0, 0.0};
    if (tid < 64) {
      if (tid < nt) dg0 = diag_term_load(H, L, tid);
      if (tid + 64 < nt) dg1 = diag_term_load(H, L, tid + 64);
    }
    const int64_t e0 = 1 + gtid;
    uint64_t ja0 = 0, jb0 = 0;
    double H0 = 0.0;
    SlotVal sv0{0, 0, 0.0, 0.0};
    SlotVal first{kEmpty, 0, 0.0, 0.0};
    int64_t slot0 = -1;
    int probes0 = 0;
    if (e0 < A.n_col) {
      H0 = column_entry(H, L, sa, sb, e0, 0.0, &ja0, &jb0);
      first = slot_load(&A.T[hash_key(ja0, jb0) & A.mask]);
    }
    if (tid < 64) {
      double part = dg0.f * (dg0.x - dg0.y) + dg1.f * (dg1.x - dg1.y);
      for (int t = tid + 128; t < nt; t += 64) part += diag_term(H, L, t);
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(part, off);
        part = (tid & off) ? (o + part) : (part + o);
      }
      if (tid == 0) {
        const double Hii = part;
        const double mud = dd_val(mu);
        const double eta = line_search(4.0 * sbv + 4.0 * mud * sc,
                                       2.0 * Hii + 4.0 * sc * sc + 2.0 * mud, 4.0 * sc);
        // mu += 2 eta c_i + eta^2 ; alpha += 2 eta b_i + eta^2 H_ii (pre-step c_i, b_i)
        dd e2 = two_prod(eta, eta);
        dd mu_n = dd_add(dd_add(mu, two_prod(2.0 * eta, sc)), e2);
        dd al_n = dd_add(dd_add(al, two_prod(2.0 * eta, sbv)), dd_mul_d(e2, Hii));
        s_bc[0] = eta;
        s_bc[1] = Hii;
        s_bc[2] = mu_n.hi;
        s_bc[3] = mu_n.lo;
        s_bc[4] = al_n.hi;
        s_bc[5] = al_n.lo;
        s_info = 0;
        s_ins_sum = 0;
        s_flags = 0;
      }
    }
    if (e0 < A.n_col) slot0 = table_find_from(A.T, A.mask, ja0, jb0, first, &probes0, &sv0);
    __syncthreads();
    const double eta = s_bc[0], Hii = s_bc[1];
    mu = dd{s_bc[2], s_bc[3]};
    al = dd{s_bc[4], s_bc[5]};
    const double mu1 = dd_val(mu);
    const double cnew = sc + eta;
    if (blockIdx.x == 0 && tid == 0) st_co(&A.T[sslot].c, cnew);

    CDFCI_TICK(tp0);
    // ---- phase B: scatter eta * H_{:,D}.  Within one iteration each b_j has a
    // single writer (the lane that owns entry j), so b_j's new value is the
    // probed value plus the increment and the atomic need not return; the
    // previous coordinate, whose correction may still be in flight, uses its
    // known recalculated value.
    Cand best{-1.0, kEmpty, kEmpty, -1, 0.0, 0.0};
    double recalc = 0.0;
    unsigned my_ins = 0;
    int err = 0;
    for (int64_t e = e0; e < A.n_col; e += gsz) {
      uint64_t ja, jb;
      double Hj;
      SlotVal sv;
      int64_t slot;
      int probes = 0;
      if (e == e0) {
        ja = ja0;
        jb = jb0;
        Hj = H0;
        sv = sv0;
        slot = slot0;
        probes = probes0;
      } else {
        Hj = column_entry(H, L, sa, sb, e, 0.0, &ja, &jb);
        slot = table_find(A.T, A.mask, ja, jb, &probes, &sv);
      }
      if (Hj == 0.0) continue;
      const double delta = eta * Hj;
      double cj = 0.0, bnew = 0.0;
      const bool is_prev = (ja == pa && jb == pb);
      if (slot >= 0) {
        cj = sv.c;
        bnew = is_prev ? pR : sv.b;
        if (cj != 0.0 || fabs(delta) >= A.tau) {
          atomic_add_f64(&A.T[slot].b, delta);
          bnew += delta;
        }
      } else if (fabs(delta) >= A.tau) {
        // the find ended at an empty slot (probes - 1 occupied ones before
        // it) unless it ran out of probes: the insert starts there
        int ins = 0;
        slot = probes < kMaxProbe
                   ? table_upsert_at(A.T, A.mask, ja, jb, (hash_key(ja, jb) + (uint64_t)(probes - 1)) & A.mask,
                                     probes - 1, &ins, &probes, &err, &sv)
                   : table_upsert(A.T, A.mask, ja, jb, &ins, &probes, &err, &sv);
        if (slot >= 0) {
          atomic_add_f64(&A.T[slot].b, delta);
          cj = sv.c;
          bnew = sv.b + delta;
          my_ins += ins;
        }
      }
      my_probe = max(my_probe, probes);
      recalc += Hj * cj;
      Cand cnd{fabs(4.0 * bnew + 4.0 * mu1 * cj), ja, jb, slot, bnew, cj};
      if (slot >= 0 && better(cnd, best)) best = cnd;
    }
    if (my_ins | err) atomicAdd(&s_info, ((unsigned long long)my_ins << 8) | (unsigned long long)err);
    block_reduce<kMaxWaves>(best, recalc, s_cand, s_sum);
    Partial* P = A.parts + (step & 1) * G;
    if (tid == 0) {
      partial_store(&P[blockIdx.x], best, recalc);
      st_co(&P[blockIdx.x].info, (int64_t)s_info);
    }
    CDFCI_TICK(tp1);
    target += G;
    if (!grid_barrier(&ctl->barrier, target)) flags |= kErrBarrier;

    CDFCI_TICK(tp2);
    // ---- phase C: combine (every workgroup, same order)
    Cand w{-1.0, kEmpty, kEmpty, -1, 0.0, 0.0};
    double rs = 0.0;
    unsigned long long ins_part = 0;  // inserts and error bits over the workgroups
    int fl_part = 0;
    for (int i = tid; i < G; i += blockDim.x) {
      double qr;
      Cand c = partial_load(&P[i], &qr);
      if (better(c, w)) w = c;
      rs += qr;
      const unsigned long long q = (unsigned long long)ld_co(&P[i].info);
      ins_part += q >> 8;
      fl_part |= (int)(q & 0xff);
    }
    if (ins_part) atomicAdd(&s_ins_sum, ins_part);
    if (fl_part) atomicOr(&s_flags, fl_part);
    block_reduce<kMaxWaves>(w, rs, s_cand, s_sum);
    const unsigned long long info = s_ins_sum;
    flags |= s_flags;
    occupied += info;
    inserts += info;
    if (occupied > A.max_entries) flags |= kErrTableFull;
    const double R = Hii * cnew + rs;
    Cand self{fabs(4.0 * R + 4.0 * mu1 * cnew), sa, sb, sslot, R, cnew};
    if (better(self, w)) w = self;
    if (blockIdx.x == 0 && tid == 0) {
      atomic_add_f64(&A.T[sslot].b, R - sbv);
      if (A.tr_E) A.tr_E[step0 + step] = dd_val(al) / mu1;
      if (A.tr_a) A.tr_a[step0 + step] = sa;
      if (A.tr_b) A.tr_b[step0 + step] = sb;
      if (A.tr_eta) A.tr_eta[step0 + step] = eta;
    }
    d = (step0 + step == 0) ? fabs(eta) : A.theta * d + (1.0 - A.theta) * fabs(eta);
    pa = sa;
    pb = sb;
    pR = R;
    sa = w.a;
    sb = w.b;
    sslot = w.slot;
    sc = w.c;
    sbv = w.bnew;
    CDFCI_TICK(tp3);
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
#undef CDFCI_TICK
  // statistics and state write-back
  __shared__ int s_probe;
  if (tid == 0) s_probe = 0;
  __syncthreads();
  atomicMax(&s_probe, my_probe);
  __syncthreads();
  if (tid == 0) atomicMax(&ctl->max_probe, s_probe);
  if (blockIdx.x == 0 && tid == 0) {
    if (flags) atomicOr(&ctl->error, flags);
    ctl->inserts += inserts;
    ctl->occupied = occupied;
    ctl->mu_hi = mu.hi;
    ctl->mu_lo = mu.lo;
    ctl->al_hi = al.hi;
    ctl->al_lo = al.lo;
    ctl->d = d;
    ctl->energy = dd_val(al) / dd_val(mu);
    ctl->sel_a = sa;
    ctl->sel_b = sb;
    ctl->sel_slot = sslot;
    ctl->sel_c = sc;
    ctl->sel_b_val = sbv;
    ctl->steps_this_call = step;
    ctl->stopped = stopped;
    ctl->t_phase[0] += tp0;
    ctl->t_phase[1] += tp1;
    ctl->t_phase[2] += tp2;
    ctl->t_phase[3] += tp3;
  }
}

// Adds the step count after the persistent kernel (one thread).
__global__ void k_finish_steps(Ctl* ctl) {
  ctl->steps += ctl->steps_this_call;
  ctl->barrier = 0;
}

__global__ void k_reset_barrier(Ctl* ctl) {
  ctl->barrier = 0;
  ctl->steps_this_call = 0;
  ctl->stopped = 0;
}

// ---------------------------------------------------------------------------
// Coulomb/exchange rows for single excitations: jk[((r*N+p)*N+k)*2] = (rp|kk),
// jk[((r*N+p)*N+k)*2+1] = (rk|kp).

// packed (pq|rs): thread t of row pq (grid y) writes the value for rs = t <= pq
__global__ void __launch_bounds__(256) k_build_eri8(const double* eri, int N, double* eri8) {
  const int npair = N * (N + 1) / 2;
  const int pq = blockIdx.y;
  if (pq >= npair) return;
  int p = 0;
  while ((p + 1) * (p + 2) / 2 <= pq) ++p;
  const int q = pq - p * (p + 1) / 2;
  for (int rs = blockIdx.x * blockDim.x + threadIdx.x; rs <= pq; rs += gridDim.x * blockDim.x) {
    int r = 0;
    while ((r + 1) * (r + 2) / 2 <= rs) ++r;
    const int s = rs - r * (r + 1) / 2;
    eri8[(int64_t)pq * (pq + 1) / 2 + rs] = eri[(((size_t)p * N + q) * N + r) * N + s];
  }
}

__global__ void __launch_bounds__(256) k_build_jk(const double* eri, int N, double* jk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)N * N * N;
  if (i >= n) return;
  const int k = (int)(i % N), p = (int)((i / N) % N), r = (int)(i / ((int64_t)N * N));
  const size_t N1 = N;
  jk[2 * i] = eri[((r * N1 + p) * N1 + k) * N1 + k];
  jk[2 * i + 1] = eri[((r * N1 + k) * N1 + k) * N1 + p];
}

// ---------------------------------------------------------------------------
// Table maintenance.

__global__ void k_shift_diag(double* h, int N, double delta) {
  for (int p = threadIdx.x; p < N; p += blockDim.x) h[p * N + p] -= delta;
}

__global__ void __launch_bounds__(256) k_clear_table(Slot* T, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    T[i] = Slot{kEmpty, kPending, 0.0, 0.0};
  }
}

__global__ void k_zero_ctl(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    uint64_t* w = reinterpret_cast<uint64_t*>(ctl);
    for (size_t i = 0; i < sizeof(Ctl) / 8; ++i) w[i] = 0;
    ctl->sel_slot = -1;
  }
}

// ---------------------------------------------------------------------------
// Initial vector: dets[0..n) with coefficients coef[0..n) are stored, then
// b = H c is scattered exactly (no compression), column by column.

struct InitTask {
  uint64_t a, b;
  double coef;
};

__global__ void k_init_insert(Slot* T, uint64_t mask, const InitTask* tasks, int n, Ctl* ctl) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int ins = 0, probes = 0, err = 0;
  SlotVal v0;
  int64_t s = table_upsert(T, mask, tasks[i].a, tasks[i].b, &ins, &probes, &err, &v0);
  if (s < 0) {
    atomicOr(&ctl->error, err ? err : kErrTableFull);
    return;
  }
  atomic_add_f64(&T[s].c, tasks[i].coef);
  if (ins) {
    atomicAdd(&ctl->occupied, 1ull);
    atomicAdd(&ctl->inserts, 1ull);
  }
}

// grid: (chunks, n tasks)
__global__ void __launch_bounds__(256) k_init_scatter(Ham H, Slot* T, uint64_t mask, const InitTask* tasks, int64_t n_col,
                               Ctl* ctl) {
  __shared__ Lists L;
  __shared__ double s_diag;
  const InitTask t = tasks[blockIdx.y];
  if (threadIdx.x == 0) {
    make_lists_serial(t.a, t.b, H.N, L);
    s_diag = diag_serial(H, L);
  }
  __syncthreads();
  unsigned long long ins_cnt = 0;
  int err = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_col;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t ja, jb;
    double Hj = column_entry(H, L, t.a, t.b, e, s_diag, &ja, &jb);
    if (Hj == 0.0) continue;
    int ins = 0, probes = 0;
    SlotVal vj;
    int64_t s = table_upsert(T, mask, ja, jb, &ins, &probes, &err, &vj);
    if (s < 0) break;
    atomic_add_f64(&T[s].b, t.coef * Hj);
    ins_cnt += ins;
  }
  if (err) atomicOr(&ctl->error, err);
  if (ins_cnt) {
    atomicAdd(&ctl->occupied, ins_cnt);
    atomicAdd(&ctl->inserts, ins_cnt);
  }
}

// mu = sum c^2, alpha = sum c b over the initial support (one workgroup,
// fixed order), then the first coordinate = argmax over all stored entries.
__global__ void k_init_scalars(const Slot* T, uint64_t mask, const InitTask* tasks, int n, Ctl* ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  dd mu{0, 0}, al{0, 0};
  for (int i = 0; i < n; ++i) {
    int probes;
    SlotVal v;
    int64_t s = table_find(T, mask, tasks[i].a, tasks[i].b, &probes, &v);
    if (s < 0) continue;
    double c = v.c, b = v.b;
    mu = dd_add(mu, two_prod(c, c));
    al = dd_add(al, two_prod(c, b));
  }
  ctl->mu_hi = mu.hi;
  ctl->mu_lo = mu.lo;
  ctl->al_hi = al.hi;
  ctl->al_lo = al.lo;
  ctl->energy = dd_val(al) / dd_val(mu);
}

// Restart from a stored wavefunction: the given entries into a cleared
// table (a key met twice is counted in *dup), then b = H c over the column of
// every entry.  With tau > 0 the stored set is the support plus every j with
// some |H_ji c_i| >= tau (pass 0 stores them), and b_j is then summed over
// all contributions (pass 1): exact on the stored set, as the compression
// rule of Sec. 3.1 keeps it for entries with c_j != 0.
__global__ void k_load_insert(Slot* T, uint64_t mask, const InitTask* tasks, int64_t n, Ctl* ctl,
                              unsigned long long* dup) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int ins = 0, probes = 0, err = 0;
  SlotVal v0;
  const int64_t s = table_upsert(T, mask, tasks[i].a, tasks[i].b, &ins, &probes, &err, &v0);
  if (s < 0) {
    atomicOr(&ctl->error, err ? err : kErrTableFull);
    return;
  }
  if (!ins) {
    atomicAdd(dup, 1ull);
    return;
  }
  st_co(&T[s].c, tasks[i].coef);
  atomicAdd(&ctl->occupied, 1ull);
  atomicAdd(&ctl->inserts, 1ull);
}

// grid: (chunks, n tasks); pass 0 stores, pass 1 accumulates
__global__ void __launch_bounds__(256) k_load_scatter(Ham H, Slot* T, uint64_t mask, const InitTask* tasks,
                                                      int64_t n_col, Ctl* ctl, double tau, int pass) {
  __shared__ Lists L;
  __shared__ double s_diag;
  const InitTask t = tasks[blockIdx.y];
  if (threadIdx.x == 0) {
    make_lists_serial(t.a, t.b, H.N, L);
    s_diag = diag_serial(H, L);
  }
  __syncthreads();
  unsigned long long ins_cnt = 0;
  int err = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_col;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t ja, jb;
    const double Hj = column_entry(H, L, t.a, t.b, e, s_diag, &ja, &jb);
    const double v = t.coef * Hj;
    if (v == 0.0) continue;
    int probes = 0;
    SlotVal vj;
    if (pass == 0) {
      if (fabs(v) < tau) continue;
      int ins = 0;
      if (table_upsert(T, mask, ja, jb, &ins, &probes, &err, &vj) < 0) break;
      ins_cnt += ins;
    } else {
      const int64_t sl = table_find(T, mask, ja, jb, &probes, &vj);
      if (sl >= 0) atomic_add_f64(&T[sl].b, v);
    }
  }
  if (err) atomicOr(&ctl->error, err);
  if (ins_cnt) {
    atomicAdd(&ctl->occupied, ins_cnt);
    atomicAdd(&ctl->inserts, ins_cnt);
  }
}

// mu = sum c^2 and alpha = sum c b over every stored entry: per-workgroup
// double-double sums (part[4 * block] = mu hi, lo, alpha hi, lo), then one
// thread over the workgroups in order
__global__ void __launch_bounds__(256) k_table_scalars(const Slot* T, uint64_t nslots, double* part) {
  __shared__ double s_red[4];
  dd mu{0.0, 0.0}, al{0.0, 0.0};
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    if (T[s].ka == kEmpty) continue;
    const double c = T[s].c, b = T[s].b;
    mu = dd_add(mu, two_prod(c, c));
    al = dd_add(al, two_prod(c, b));
  }
  const dd m = wg_sum_dd(mu, s_red);
  const dd a = wg_sum_dd(al, s_red);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = m.hi;
    part[4 * blockIdx.x + 1] = m.lo;
    part[4 * blockIdx.x + 2] = a.hi;
    part[4 * blockIdx.x + 3] = a.lo;
  }
}

__global__ void k_table_scalars_final(const double* part, int nb, Ctl* ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  dd mu{0.0, 0.0}, al{0.0, 0.0};
  for (int i = 0; i < nb; ++i) {
    mu = dd_add(mu, dd{part[4 * i], part[4 * i + 1]});
    al = dd_add(al, dd{part[4 * i + 2], part[4 * i + 3]});
  }
  ctl->mu_hi = mu.hi;
  ctl->mu_lo = mu.lo;
  ctl->al_hi = al.hi;
  ctl->al_lo = al.lo;
  ctl->energy = dd_val(al) / dd_val(mu);
}

// argmax of |4b + 4 mu c| over every stored entry (used once after init)
__global__ void __launch_bounds__(256) k_select_table(const Slot* T, uint64_t nslots, Ctl* ctl, Partial* parts) {
  __shared__ Cand s_cand[kMaxWaves];
  __shared__ double s_sum[kMaxWaves];
  const double mu = ctl->mu_hi + ctl->mu_lo;
  Cand best{-1.0, kEmpty, kEmpty, -1, 0.0, 0.0};
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    Slot s = T[i];
    if (s.ka == kEmpty) continue;
    Cand c{fabs(4.0 * s.b + 4.0 * mu * s.c), s.ka, s.kb, (int64_t)i, s.b, s.c};
    if (better(c, best)) best = c;
  }
  double dummy = 0.0;
  block_reduce<kMaxWaves>(best, dummy, s_cand, s_sum);
  if (threadIdx.x == 0)
    parts[blockIdx.x] = Partial{best.g, best.a, best.b, best.slot, best.bnew, best.c, 0.0, 0};
}

__global__ void k_select_final(const Partial* parts, int n, Ctl* ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Cand w{-1.0, kEmpty, kEmpty, -1, 0.0, 0.0};
  for (int i = 0; i < n; ++i) {
    Cand c{parts[i].g, parts[i].a, parts[i].b, parts[i].slot, parts[i].bnew, parts[i].c};
    if (better(c, w)) w = c;
  }
  ctl->sel_a = w.a;
  ctl->sel_b = w.b;
  ctl->sel_slot = w.slot;
  ctl->sel_c = w.c;
  ctl->sel_b_val = w.bnew;
}

// ---------------------------------------------------------------------------
// Subspace initial vector (lattice models): D0 plus the nonzero entries of its
// column; H on that set; lowest eigenpair by cyclic Jacobi (one thread).

constexpr int kMaxSub = 128;

// One workgroup of 256 threads.  Tasks: D0, then the nonzero entries of its
// column in enumeration order (an order-preserving compaction); A on them;
// cyclic Jacobi in the parallel (round-robin) ordering: each round rotates
// n/2 disjoint index pairs at once, which is the same transform as applying
// those rotations one after another (disjoint planes commute, and each
// rotation's 2 x 2 block depends on its own rows and columns only).
__global__ void __launch_bounds__(256) k_subspace_init(Ham H, uint64_t a0, uint64_t b0, int64_t n_col,
                                                       InitTask* out, int* n_out,
                                                       double* work /* kMaxSub^2 * 2 */, int* status) {
  __shared__ Lists L;
  __shared__ double s_red[4];
  __shared__ int s_n, s_wave[4];
  __shared__ double s_c[kMaxSub / 2], s_s[kMaxSub / 2];
  __shared__ int s_p[kMaxSub / 2], s_q[kMaxSub / 2];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  make_lists_block(a0, b0, H.N, L);
  __syncthreads();
  double part = 0.0;
  const int nt = diag_terms(L);
  for (int t = tid; t < nt; t += blockDim.x) part += diag_term(H, L, t);
  const double d0 = wg_sum(part, s_red);
  if (tid == 0) {
    out[0] = InitTask{a0, b0, 0.0};
    s_n = 1;
  }
  __syncthreads();
  for (int64_t base = 1; base < n_col; base += blockDim.x) {
    const int64_t e = base + tid;
    uint64_t ja = 0, jb = 0;
    double v = 0.0;
    if (e < n_col) v = column_entry(H, L, a0, b0, e, d0, &ja, &jb);
    const bool nz = e < n_col && v != 0.0;
    const unsigned long long bal = __ballot(nz);
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[wv] = __popcll(bal);
    __syncthreads();
    int pos = s_n + below;
    for (int q = 0; q < wv; ++q) pos += s_wave[q];
    if (nz && pos < kMaxSub) out[pos] = InitTask{ja, jb, 0.0};
    __syncthreads();
    if (tid == 0) s_n += s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
  }
  const int n = s_n;
  if (n > kMaxSub) {
    if (tid == 0) *status = -2;
    return;
  }
  double* A = work;
  double* V = work + kMaxSub * kMaxSub;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    Lists Lj;
    make_lists_serial(out[j].a, out[j].b, H.N, Lj);
    const double dj = (i == j) ? diag_serial(H, Lj) : 0.0;
    A[i * n + j] = sc_entry(H, out[i].a, out[i].b, out[j].a, out[j].b, Lj, dj);
    V[i * n + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int m2 = n + (n & 1);  // even number of positions; position n (if any) is idle
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    double o = 0.0;
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
      const int i = idx / n, j = idx % n;
      if (i < j) o += A[idx] * A[idx];
    }
    o = wg_sum(o, s_red);
    if (o < 1e-30) break;
    for (int r = 0; r < m2 - 1; ++r) {
      if (tid < m2 / 2) {
        // round-robin pairing: position 0 fixed, the others rotate
        const int k = tid;
        const int x = k == 0 ? 0 : 1 + (k - 1 + r) % (m2 - 1);
        const int y = 1 + (m2 - 2 - k + r) % (m2 - 1);
        int p = x < y ? x : y, q = x < y ? y : x;
        double c = 1.0, sn = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          if (apq != 0.0) {
            const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
          }
        } else {
          p = q = -1;
        }
        s_p[k] = p;
        s_q[k] = q;
        s_c[k] = c;
        s_s[k] = sn;
      }
      __syncthreads();
      const int np = m2 / 2;
      // A <- J^T A: rows p, q of every pair
      for (int idx = tid; idx < np * n; idx += blockDim.x) {
        const int k = idx / n, col = idx % n, p = s_p[k], q = s_q[k];
        if (p < 0 || s_s[k] == 0.0) continue;
        const double c = s_c[k], sn = s_s[k];
        const double apk = A[p * n + col], aqk = A[q * n + col];
        A[p * n + col] = c * apk - sn * aqk;
        A[q * n + col] = sn * apk + c * aqk;
      }
      __syncthreads();
      // A <- A J and V <- V J: columns p, q of every pair
      for (int idx = tid; idx < np * n; idx += blockDim.x) {
        const int k = idx / n, row = idx % n, p = s_p[k], q = s_q[k];
        if (p < 0 || s_s[k] == 0.0) continue;
        const double c = s_c[k], sn = s_s[k];
        const double akp = A[row * n + p], akq = A[row * n + q];
        A[row * n + p] = c * akp - sn * akq;
        A[row * n + q] = sn * akp + c * akq;
        const double vkp = V[row * n + p], vkq = V[row * n + q];
        V[row * n + p] = c * vkp - sn * vkq;
        V[row * n + q] = sn * vkp + c * vkq;
      }
      __syncthreads();
    }
  }
  if (tid != 0) return;
  int m = 0;
  for (int i = 1; i < n; ++i)
    if (A[i * n + i] < A[m * n + m]) m = i;
  const double lam = A[m * n + m];
  if (!(lam < 0.0)) {
    *status = -4;
    return;
  }
  const double sgn = V[0 * n + m] < 0.0 ? -1.0 : 1.0;
  const double scale = sqrt(-lam) * sgn;
  for (int i = 0; i < n; ++i) out[i].coef = scale * V[i * n + m];
  *n_out = n;
  *status = 0;
}

// Aufbau determinant on the device: the n lowest h_pp (ties: lower index).
__global__ void k_aufbau_init(Ham H, InitTask* out, int* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t used = 0, a = 0, b = 0;
  for (int k = 0; k < max(H.na, H.nb); ++k) {
    int best = -1;
    for (int p = 0; p < H.N; ++p) {
      if ((used >> p) & 1) continue;
      if (best < 0 || H.h[p * H.N + p] < H.h[best * H.N + best]) best = p;
    }
    used |= 1ull << best;
    if (k < H.na) a |= 1ull << best;
    if (k < H.nb) b |= 1ull << best;
  }
  Lists L;
  make_lists_serial(a, b, H.N, L);
  double d0 = diag_serial(H, L);
  if (!(d0 < 0.0)) {
    *status = -4;
    return;
  }
  out[0] = InitTask{a, b, sqrt(-d0)};
  *status = 0;
}

// ---------------------------------------------------------------------------
// Inspection kernels.

// diag_shift is added to the diagonal entry (the context holds H - sigma I;
// get_column reports H)
__global__ void __launch_bounds__(256) k_column(Ham H, uint64_t a, uint64_t b, int64_t n_col, double diag_shift,
                                                uint64_t* keys, double* vals) {
  __shared__ Lists L;
  __shared__ double s_diag;
  if (threadIdx.x == 0) {
    make_lists_serial(a, b, H.N, L);
    s_diag = diag_serial(H, L) + diag_shift;
  }
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_col;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t ja, jb;
    double v = column_entry(H, L, a, b, e, s_diag, &ja, &jb);
    keys[2 * e] = ja;
    keys[2 * e + 1] = jb;
    vals[e] = v;
  }
}

__global__ void k_entry(Ham H, uint64_t a1, uint64_t b1, uint64_t a2, uint64_t b2, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Lists L;
  make_lists_serial(a2, b2, H.N, L);
  double d = diag_serial(H, L);
  *out = sc_entry(H, a1, b1, a2, b2, L, d);
}

// Random-access calibration (cdfci_random_access_rates): the memory
// operations the column scatter is made of, each on its own over uniformly
// random slots of a table as large as the solver's.  Only the timing matters;
// the values written are meaningless.
__global__ void __launch_bounds__(256) k_ra_fill(Slot* T, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    T[i].ka = hash_key(i, 1);
    T[i].kb = hash_key(i, 2);
    T[i].c = 0.0;
    T[i].b = 0.0;
  }
}
// kind 0: 16-byte key gather; 1: gather and plain read-modify-write of b;
// 2: gather and agent-scope FP64 atomic add to b; 3: returning atomic OR into
// a bitmap of one bit per slot
__global__ void __launch_bounds__(256) k_ra(Slot* T, unsigned* bitmap, uint64_t mask, uint64_t n, uint64_t salt,
                                            int kind, unsigned long long* sink) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t idx = hash_key(i, salt) & mask;
  uint64_t acc = 0;
  if (kind == 3) {
    acc = atomicOr(&bitmap[idx >> 5], 1u << (idx & 31));
  } else {
    const ulonglong2 kk = *reinterpret_cast<const ulonglong2*>(&T[idx]);
    acc = kk.x ^ kk.y;
    if (kind == 1 && acc != 1) T[idx].b = T[idx].b + 1.0;
    if (kind == 2 && acc != 1) atomic_add_f64(&T[idx].b, 1.0);
  }
  if (acc == 1) *sink = acc;  // keeps the loads
}
__global__ void __launch_bounds__(256) k_ra_copy(const double4* a, double4* b, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// compact occupied slots (c != 0 if nonzero_c) into a list of slot ids
__global__ void __launch_bounds__(256) k_compact(const Slot* T, uint64_t nslots, int nonzero_c, int64_t* list,
                          unsigned long long* count, int64_t cap) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    Slot s = T[i];
    if (s.ka == kEmpty) continue;
    if (nonzero_c && s.c == 0.0) continue;
    unsigned long long k = atomicAdd(count, 1ull);
    if ((int64_t)k < cap) list[k] = (int64_t)i;
  }
}

__global__ void __launch_bounds__(256) k_gather(const Slot* T, const int64_t* list, int64_t n, uint64_t* keys, double* c,
                         double* b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    Slot s = T[list[i]];
    keys[2 * i] = s.ka;
    keys[2 * i + 1] = s.kb;
    c[i] = s.c;
    b[i] = s.b;
  }
}

// c^T H c over the support: each workgroup takes support determinants in turn
// and sums c_i H_ji c_j over the column of i; per-workgroup partial sums.
__global__ void __launch_bounds__(256) k_apply_energy(Ham H, const Slot* T, uint64_t mask, const int64_t* list, int64_t n,
                               int64_t n_col, double* partial_num, double* partial_den) {
  __shared__ Lists L;
  __shared__ double s_diag;
  __shared__ Cand s_cand[kMaxWaves];
  __shared__ double s_sum[kMaxWaves];
  double num = 0.0, den = 0.0;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    Slot si = T[list[i]];
    __syncthreads();
    if (threadIdx.x == 0) {
      make_lists_serial(si.ka, si.kb, H.N, L);
      s_diag = diag_serial(H, L);
    }
    __syncthreads();
    if (threadIdx.x == 0) den += si.c * si.c;
    for (int64_t e = threadIdx.x; e < n_col; e += blockDim.x) {
      uint64_t ja, jb;
      double v = column_entry(H, L, si.ka, si.kb, e, s_diag, &ja, &jb);
      if (v == 0.0) continue;
      int probes;
      SlotVal sv;
      int64_t s = table_find(T, mask, ja, jb, &probes, &sv);
      if (s < 0) continue;
      num += si.c * v * sv.c;
    }
  }
  Cand dummy{0, 0, 0, 0, 0, 0};
  block_reduce<kMaxWaves>(dummy, num, s_cand, s_sum);
  block_reduce<kMaxWaves>(dummy, den, s_cand, s_sum);
  if (threadIdx.x == 0) {
    partial_num[blockIdx.x] = num;
    partial_den[blockIdx.x] = den;
  }
}

__global__ void k_sum_partials(const double* num, const double* den, int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  dd a{0, 0}, b{0, 0};
  for (int i = 0; i < n; ++i) {
    a = dd_add(a, dd{num[i], 0.0});
    b = dd_add(b, dd{den[i], 0.0});
  }
  out[0] = dd_val(a);
  out[1] = dd_val(b);
}

#include "mcd_kernels.h"
#include "rdm_kernels.h"
#include "hub_kernels.h"
#include "xcd_kernels.h"
#include "orb_kernels.h"

// per-instance step budget of the coming wave: the listed (resident)
// instances may advance nsteps iterations
__global__ void k_hub_limits(HubInst* inst, const unsigned* ids, int n, int64_t nsteps) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  HubInst& P = inst[ids[k]];
  P.step_limit = P.ctl->steps + nsteps;
}

struct HubResult {
  double energy;
  int64_t steps;
  unsigned long long elements, occupied;
  int stopped, error;
};

// results of the listed (resident) instances, in list order
__global__ void k_hub_results(const HubInst* inst, const unsigned* ids, int n, HubResult* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const HubInst& P = inst[ids[k]];
  const Ctl* c = P.ctl;
  out[k] = HubResult{(c->al_hi + c->al_lo) / (c->mu_hi + c->mu_lo), c->steps, *P.elements,
                     c->occupied, c->stopped, c->error};
}

}  // namespace

// ===========================================================================
// Host side.

struct cdfci_ctx {
  int N, na, nb;
  int device;
  hipStream_t stream;
  double* d_h = nullptr;
  double* d_eri = nullptr;
  double* d_eri8 = nullptr;
  double* d_jk = nullptr;
  Slot* T = nullptr;
  uint64_t nslots = 0, mask = 0, max_entries = 0;
  bool own_table = false;
  Ctl* ctl = nullptr;
  Partial* parts = nullptr;
  int max_parts = 0;
  int64_t n_col = 0;
  cdfci_opts opts;
  double shift = 0.0;  // sigma of opts.energy_shift: the device holds H - sigma I
  int grid = 0, block = 256;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool poisoned = false;
  // scratch for inspection/energy calls
  int64_t* list = nullptr;
  int64_t list_cap = 0;
  double* dscratch = nullptr;  // 2 * 2048 partials + 2
  // multicoordinate state (allocated on the first k > 1 step)
  int mode = 0;  // 0: single-coordinate state current, 1: multicoordinate state current
  int mc_kcap = 0;
  uint64_t cand_cap = 0;
  McState* mst = nullptr;
  unsigned* cand = nullptr;  // candidate pages (kPage slot ids each)
  unsigned* cnt = nullptr;   // entries used per page
  unsigned long long* pkey = nullptr;  // selection key of every candidate position (cand_cap)
  unsigned long long* gkey = nullptr;  // dense selection keys (cand_cap + one grid of slack)
  unsigned* dslot = nullptr;           // dense selection slots
  unsigned* dcount = nullptr;          // dense region lengths (kSelBlocks)
  unsigned* ties = nullptr;            // keys equal to the threshold (grid gather, kMaxTies)
  unsigned* hist = nullptr;
  int64_t* sel_slot = nullptr;
  uint64_t* sel_a = nullptr;
  uint64_t* sel_b = nullptr;
  double* eta = nullptr;
  PageStat* pstat = nullptr;  // per scatter workgroup: recalculation part and counts
  uint64_t pstat_cap = 0;
  // per-phase device time of multicoordinate steps (cdfci_set_timing)
  int timing = 0;
  std::vector<hipEvent_t> tev;
  // select, H_II, reduced problem with the probe half, apply half, finish; probe half alone
  double t_phase_mc[7] = {0, 0, 0, 0, 0, 0, 0};
  int64_t n_timed = 0;
  unsigned long long* ptime = nullptr;  // probe-half and solver timestamps, 4 per timed step
  int64_t ptime_cap = 0;
  double* hii = nullptr;
  double* chat = nullptr;       // c_hat of the chosen set after a step
  ScatRec* rec = nullptr;       // probe-half records, one per column entry of each chosen column
  unsigned* bitmap = nullptr;   // one bit per slot, clear between selections (bm_words words)
  uint64_t bm_words = 0;
};

struct cdfci_batch {
  int count = 0;
  std::vector<cdfci_hubbard_spec> specs;
  std::vector<cdfci_ctx*> ctx;              // resident instances (nullptr otherwise)
  std::vector<uint64_t> slots;              // planned table slots per instance
  std::vector<HubInst> h_inst;              // host copy of the per-instance kernel arguments
  std::vector<HubResult> res;               // last known results (steps counted since init)
  std::vector<int> init_error;              // CDFCI_ERR_* of an instance whose start failed
  std::vector<int64_t> base_steps;          // iterations before the last restart
  std::vector<std::vector<uint64_t>> ck_keys;  // checkpoint of an evicted running instance
  std::vector<std::vector<double>> ck_c;
  uint64_t budget = 0, resident = 0, peak = 0;  // resident: table memory held (in use or pooled)
  std::vector<std::pair<uint64_t, void*>> pool;  // released tables kept for the next admission
  std::vector<void*> table_of;                   // table buffer of each resident instance
  int restarts = 0;
  HubInst* d_inst = nullptr;
  unsigned* d_active = nullptr;
  unsigned* d_queue = nullptr;
  unsigned long long* d_elems = nullptr;
  HubResult* d_res = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_n = -1, graph_waves = -1;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  cdfci_batch_opts opts;
  int waves = 0;
};

namespace {

Ham ham_of(const cdfci_ctx* c) { return Ham{c->N, c->na, c->nb, c->d_h, c->d_eri8, c->d_jk}; }

int ctl_read(cdfci_ctx* c, Ctl* host) {
  HIP_TRY(hipMemcpyAsync(host, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return 0;
}

int check_error(cdfci_ctx* c, const Ctl& h) {
  if (h.error & kErrTableFull) {
    c->poisoned = true;
    return CDFCI_ERR_TABLE_FULL;
  }
  if (h.error & kErrBarrier) {
    c->poisoned = true;
    return CDFCI_ERR_BARRIER;
  }
  if (h.error & kErrPublish) {
    c->poisoned = true;
    return CDFCI_ERR_HIP;
  }
  if (h.error & kErrNumeric) {
    c->poisoned = true;
    return CDFCI_ERR_NUMERIC;
  }
  if (h.error & kErrSelect) {
    c->poisoned = true;
    g_last_error = "a multicoordinate selection's bound held fewer than k distinct determinants";
    return CDFCI_ERR_INTERNAL;
  }
  if (h.occupied > c->max_entries) {
    c->poisoned = true;
    return CDFCI_ERR_TABLE_FULL;
  }
  return 0;
}

void fill_defaults(cdfci_opts& o) {
  if (o.table_slots == 0) o.table_slots = 1ull << 22;
  if (o.load_factor <= 0.0) o.load_factor = 0.79;
  if (o.dx_damping <= 0.0) o.dx_damping = 0.9;
  if (o.block_threads < 0) o.block_threads = 0;  // 0: chosen from the column size at set-up
}

int ensure_list(cdfci_ctx* c, int64_t n) {
  if (c->list_cap >= n) return 0;
  if (c->list) HIP_TRY(hipFree(c->list));
  c->list = nullptr;
  int64_t cap = std::max<int64_t>(n, 1024);
  HIP_TRY(hipMalloc(&c->list, cap * sizeof(int64_t)));
  c->list_cap = cap;
  return 0;
}

// common setup after integrals are on the device
int setup_and_init(cdfci_ctx* c, int init_kind, uint64_t neel_a, uint64_t neel_b) {
  const cdfci_opts& o = c->opts;
  c->nslots = o.table_slots;
  c->mask = c->nslots - 1;
  c->max_entries = (uint64_t)(o.load_factor * (double)c->nslots);
  size_t tbytes = c->nslots * sizeof(Slot);
  if (o.workspace) {
    if (o.workspace_bytes < tbytes || ((uintptr_t)o.workspace & 255)) return CDFCI_ERR_WORKSPACE;
    c->T = (Slot*)o.workspace;
    c->own_table = false;
  } else {
    HIP_TRY(hipMalloc(&c->T, tbytes));
    c->own_table = true;
  }
  HIP_TRY(hipMalloc(&c->ctl, sizeof(Ctl)));
  c->max_parts = 4096;
  HIP_TRY(hipMalloc(&c->parts, 2 * c->max_parts * sizeof(Partial)));
  HIP_TRY(hipMalloc(&c->dscratch, (2 * 4096 + 8) * sizeof(double)));
  HIP_TRY(hipEventCreate(&c->ev0));
  HIP_TRY(hipEventCreate(&c->ev1));
  c->n_col = column_count(c->N, c->na, c->nb);

  // persistent grid: enough lanes for one column entry each, bounded by residency
  int dev_cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device));
  // automatic workgroup size: 128 threads while the column still gives every
  // lane one entry within one workgroup per compute unit (a shorter tail of
  // slow probes per workgroup), else 256
  if (c->block == 0) c->block = (c->n_col + 127) / 128 <= dev_cus ? 128 : 256;
  int per_cu = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_cd1, c->block, 0));
  int max_grid = std::max(1, per_cu) * dev_cus;
  int want = o.grid_blocks > 0 ? o.grid_blocks
                               : (int)std::min<int64_t>((c->n_col + c->block - 1) / c->block, dev_cus);
  c->grid = std::max(1, std::min(want, std::min(max_grid, c->max_parts)));

  hipStream_t s = c->stream;
  k_zero_ctl<<<1, 1, 0, s>>>(c->ctl);
  k_clear_table<<<2048, 256, 0, s>>>(c->T, c->nslots);
  HIP_TRY(hipGetLastError());

  InitTask* d_tasks = nullptr;
  int* d_stat = nullptr;
  int* d_n = nullptr;
  double* d_work = nullptr;
  HIP_TRY(hipMalloc(&d_tasks, kMaxSub * sizeof(InitTask)));
  HIP_TRY(hipMalloc(&d_stat, 2 * sizeof(int)));
  int ntask = 1;
  int rc = 0;
  Ham H = ham_of(c);
  if (init_kind == 2) {
    HIP_TRY(hipMalloc(&d_work, 2 * kMaxSub * kMaxSub * sizeof(double)));
    d_n = d_stat + 1;
    k_subspace_init<<<1, 256, 0, s>>>(H, neel_a, neel_b, c->n_col, d_tasks, d_n, d_work, d_stat);
  } else {
    k_aufbau_init<<<1, 1, 0, s>>>(H, d_tasks, d_stat);
  }
  HIP_TRY(hipGetLastError());
  int hstat[2] = {0, 1};
  HIP_TRY(hipMemcpyAsync(hstat, d_stat, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hstat[0] == -4) rc = CDFCI_ERR_NOT_NEGATIVE;
  else if (hstat[0] != 0) rc = CDFCI_ERR_UNSUPPORTED;
  if (init_kind == 2 && rc == 0) ntask = hstat[1];
  if (rc == 0) {
    k_init_insert<<<(ntask + 63) / 64, 64, 0, s>>>(c->T, c->mask, d_tasks, ntask, c->ctl);
    int chunks = (int)std::min<int64_t>((c->n_col + 255) / 256, 1024);
    k_init_scatter<<<dim3(chunks, ntask), 256, 0, s>>>(H, c->T, c->mask, d_tasks, c->n_col, c->ctl);
    k_init_scalars<<<1, 1, 0, s>>>(c->T, c->mask, d_tasks, ntask, c->ctl);
    int sel_blocks = (int)std::min<uint64_t>((c->nslots + 255) / 256, (uint64_t)c->max_parts);
    k_select_table<<<sel_blocks, 256, 0, s>>>(c->T, c->nslots, c->ctl, c->parts);
    k_select_final<<<1, 1, 0, s>>>(c->parts, sel_blocks, c->ctl);
    HIP_TRY(hipGetLastError());
    Ctl h;
    int e = ctl_read(c, &h);
    if (e) rc = e;
    else rc = check_error(c, h);
  }
  (void)hipFree(d_tasks);
  (void)hipFree(d_stat);
  if (d_work) (void)hipFree(d_work);
  return rc;
}

int make_ctx(int N, int na, int nb, const cdfci_opts* opts, cdfci_ctx** out) {
  if (!out) return CDFCI_ERR_INVALID_ARG;
  *out = nullptr;
  if (N < 1 || N > kMaxOrb || na < 0 || nb < 0 || na > N || nb > N) return CDFCI_ERR_UNSUPPORTED;
  if (na + nb < 1) return CDFCI_ERR_INVALID_ARG;
  cdfci_opts o;
  memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  fill_defaults(o);
  if ((o.table_slots & (o.table_slots - 1)) != 0 || o.table_slots < 64) return CDFCI_ERR_INVALID_ARG;
  if (o.block_threads % 64 != 0 || o.block_threads > 256) return CDFCI_ERR_INVALID_ARG;
  if (o.load_factor > 0.95) return CDFCI_ERR_INVALID_ARG;
  if (!std::isfinite(o.energy_shift)) return CDFCI_ERR_INVALID_ARG;
  cdfci_ctx* c = new cdfci_ctx();
  c->shift = o.energy_shift;
  c->N = N;
  c->na = na;
  c->nb = nb;
  c->opts = o;
  c->block = o.block_threads;
  c->stream = (hipStream_t)o.stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return CDFCI_ERR_HIP;
  }
  {
    hipError_t e = resolve_scratch(c->device);
    if (e != hipSuccess) {
      g_last_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      delete c;
      return CDFCI_ERR_HIP;
    }
  }
  *out = c;
  return 0;
}

int upload(cdfci_ctx* c, const double* h, const double* eri) {
  size_t N = c->N;
  HIP_TRY(hipMalloc(&c->d_h, N * N * sizeof(double)));
  HIP_TRY(hipMalloc(&c->d_eri, N * N * N * N * sizeof(double)));
  // host or device sources (unified addressing picks the direction)
  HIP_TRY(hipMemcpyAsync(c->d_h, h, N * N * sizeof(double), hipMemcpyDefault, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_eri, eri, N * N * N * N * sizeof(double), hipMemcpyDefault, c->stream));
  // energy shift: h - (sigma / n) I is H - sigma I on the n-electron space
  if (c->shift != 0.0)
    k_shift_diag<<<1, 64, 0, c->stream>>>(c->d_h, c->N, c->shift / (double)(c->na + c->nb));
  HIP_TRY(hipMalloc(&c->d_jk, 2 * N * N * N * sizeof(double)));
  const int64_t njk = (int64_t)N * N * N;
  k_build_jk<<<(int)((njk + 255) / 256), 256, 0, c->stream>>>(c->d_eri, c->N, c->d_jk);
  const int npair = (int)(N * (N + 1) / 2);
  HIP_TRY(hipMalloc(&c->d_eri8, (size_t)npair * (npair + 1) / 2 * sizeof(double)));
  k_build_eri8<<<dim3((npair + 255) / 256, npair), 256, 0, c->stream>>>(c->d_eri, c->N, c->d_eri8);
  HIP_TRY(hipGetLastError());
  return 0;
}

std::vector<std::pair<int, int>> lattice_bonds(const int* dims, int ndim) {
  int L = 1;
  for (int i = 0; i < ndim; ++i) L *= dims[i];
  std::vector<std::pair<int, int>> bonds;
  std::vector<int> coord(ndim);
  for (int site = 0; site < L; ++site) {
    int rem = site;
    for (int ax = ndim - 1; ax >= 0; --ax) {
      coord[ax] = rem % dims[ax];
      rem /= dims[ax];
    }
    for (int ax = 0; ax < ndim; ++ax) {
      if (dims[ax] < 2) continue;
      std::vector<int> nb = coord;
      nb[ax] = (nb[ax] + 1) % dims[ax];
      int other = 0;
      for (int k = 0; k < ndim; ++k) other = other * dims[k] + nb[k];
      if (other == site) continue;
      std::pair<int, int> bd(std::min(site, other), std::max(site, other));
      if (std::find(bonds.begin(), bonds.end(), bd) == bonds.end()) bonds.push_back(bd);
    }
  }
  return bonds;
}

// Periodic Hubbard lattice as integrals: -t on each distinct bond, (ii|ii) = U.
void hubbard_integrals(const int* dims, int ndim, double t, double U, std::vector<double>& h,
                       std::vector<double>& eri) {
  int L = 1;
  for (int i = 0; i < ndim; ++i) L *= dims[i];
  h.assign((size_t)L * L, 0.0);
  eri.assign((size_t)L * L * L * L, 0.0);
  for (auto& bd : lattice_bonds(dims, ndim)) {
    h[(size_t)bd.first * L + bd.second] = -t;
    h[(size_t)bd.second * L + bd.first] = -t;
  }
  for (int i = 0; i < L; ++i) eri[(((size_t)i * L + i) * L + i) * L + i] = U;
}

// Neel determinant: alpha on the even-coordinate-sum sublattice (then the
// rest), beta on the remaining sites (then the alpha sites), ascending.
void neel_determinant(const int* dims, int ndim, int n_alpha, int n_beta, uint64_t* a0, uint64_t* b0) {
  int L = 1;
  for (int i = 0; i < ndim; ++i) L *= dims[i];
  std::vector<int> even, odd;
  for (int site = 0; site < L; ++site) {
    int rem = site, sum = 0;
    for (int ax = ndim - 1; ax >= 0; --ax) {
      sum += rem % dims[ax];
      rem /= dims[ax];
    }
    (sum % 2 == 0 ? even : odd).push_back(site);
  }
  std::vector<int> order = even;
  order.insert(order.end(), odd.begin(), odd.end());
  uint64_t a = 0, b = 0;
  for (int k = 0; k < n_alpha; ++k) a |= 1ull << order[k];
  std::vector<int> rest;
  for (int site = 0; site < L; ++site)
    if (!((a >> site) & 1)) rest.push_back(site);
  for (int site = 0; site < L; ++site)
    if ((a >> site) & 1) rest.push_back(site);
  for (int k = 0; k < n_beta; ++k) b |= 1ull << rest[k];
  *a0 = a;
  *b0 = b;
}

// device buffers owned by one library call, released when it returns
// (hipFree waits for the work that uses them)
struct CallBufs {
  std::vector<void*> ptrs;
  ~CallBufs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t alloc(T** out, uint64_t n) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<uint64_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(p);
    *out = (T*)p;
    return e;
  }
};

// Slot ids of the top_n stored determinants by |c| (equal |c| ordered by the
// smaller key), or of every entry with c != 0 when top_n <= 0 or exceeds that
// count, into *sel (device, owned by bufs); the count into *n_out.  Uses the
// radix select of the multicoordinate step keyed on |c|.
int select_support(cdfci_ctx* c, int64_t top_n, CallBufs& bufs, int64_t** sel, int64_t* n_out) {
  hipStream_t s = c->stream;
  if (c->mode == 1) {  // true values: fold the multicoordinate lazy scale in
    k_mc_rescale<<<2048, 256, 0, s>>>(c->T, c->nslots, c->mst, 1);
    k_mc_rescale_done<<<1, 1, 0, s>>>(c->mst, 1);
  }
  Ctl h;
  int rc = ctl_read(c, &h);
  if (rc) return rc;
  const uint64_t pages = (h.occupied + kPage) / kPage;
  const uint64_t cap = pages * kPage;
  McState* st;
  unsigned *cand, *cnt, *hist, *ties;
  unsigned long long* gkey;
  unsigned *dslot, *dcount;
  HIP_TRY(bufs.alloc(&st, 1));
  HIP_TRY(bufs.alloc(&cand, cap));
  HIP_TRY(bufs.alloc(&cnt, pages));
  HIP_TRY(bufs.alloc(&gkey, cap + (uint64_t)kSelBlocks * kPage));
  HIP_TRY(bufs.alloc(&dslot, cap + (uint64_t)kSelBlocks * kPage));
  HIP_TRY(bufs.alloc(&dcount, kSelBlocks));
  HIP_TRY(bufs.alloc(&hist, kRadixBins));
  HIP_TRY(bufs.alloc(&ties, kMaxTies));
  HIP_TRY(hipMemsetAsync(st, 0, sizeof(McState), s));
  HIP_TRY(hipMemsetAsync(hist, 0, kRadixBins * sizeof(unsigned), s));
  k_rdm_nonzero<<<2048, 256, 0, s>>>(c->T, c->nslots, cand, st, cap);
  HIP_TRY(hipGetLastError());
  unsigned long long nnz = 0;
  HIP_TRY(hipMemcpyAsync(&nnz, &st->n_dense, sizeof(nnz), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (nnz == 0 || nnz > cap) return CDFCI_ERR_INVALID_ARG;
  const int64_t n = (top_n > 0 && (uint64_t)top_n < nnz) ? top_n : (int64_t)nnz;
  if (n > (int64_t)0x7fffffff) return CDFCI_ERR_UNSUPPORTED;
  k_mc_dense_pages<<<256, 256, 0, s>>>(cnt, st, cap);
  uint64_t *sa, *sb;
  HIP_TRY(bufs.alloc(sel, n));
  HIP_TRY(bufs.alloc(&sa, n));
  HIP_TRY(bufs.alloc(&sb, n));
  for (int pass = 0; pass < kRadixPasses; ++pass)
    k_mc_radix<<<kSelBlocks, 256, 0, s>>>(c->T, cand, cnt, SelBufs{gkey, dslot, dcount}, c->ctl, st, hist, pass, 1,
                                          (int)n);
  k_mc_gather_ties<<<kSelBlocks, 256, 0, s>>>(c->T, SelBufs{gkey, dslot, dcount}, st, *sel, ties, sa, sb, (int)n,
                                              nullptr);
  HIP_TRY(hipGetLastError());
  unsigned long long got = 0;
  HIP_TRY(hipMemcpyAsync(&got, &st->n_sel, sizeof(got), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  // more than kMaxTies entries of exactly the threshold |c| are not ranked
  if ((int64_t)got != n) return CDFCI_ERR_UNSUPPORTED;
  *n_out = n;
  return 0;
}

}  // namespace

extern "C" {

int cdfci_workspace_size(int n_orb, int n_alpha, int n_beta, const cdfci_opts* opts, size_t* bytes) {
  if (!bytes) return CDFCI_ERR_INVALID_ARG;
  if (n_orb < 1 || n_orb > kMaxOrb || n_alpha > n_orb || n_beta > n_orb) return CDFCI_ERR_UNSUPPORTED;
  cdfci_opts o;
  memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  fill_defaults(o);
  *bytes = o.table_slots * sizeof(Slot);
  return 0;
}

int cdfci_init(const double* h, const double* eri, int n_orb, int n_alpha, int n_beta,
               const cdfci_opts* opts, cdfci_ctx** out) {
  if (!h || !eri) return CDFCI_ERR_INVALID_ARG;
  int rc = make_ctx(n_orb, n_alpha, n_beta, opts, out);
  if (rc) return rc;
  cdfci_ctx* c = *out;
  rc = upload(c, h, eri);
  int kind = c->opts.init_kind == 2 ? 2 : 1;
  uint64_t a0 = 0, b0 = 0;
  if (!rc && kind == 2) {
    // lowest-index Neel pattern for a chain: alternate sites
    for (int p = 0, ka = 0; p < n_orb && ka < n_alpha; p += 2, ++ka) a0 |= 1ull << p;
    for (int p = 1, kb = 0; p < n_orb && kb < n_beta; p += 2, ++kb) b0 |= 1ull << p;
  }
  if (!rc) rc = setup_and_init(c, kind, a0, b0);
  if (rc) {
    cdfci_free(c);
    *out = nullptr;
  }
  return rc;
}

int cdfci_init_hubbard(const int* dims, int ndim, double t, double U, int n_alpha, int n_beta,
                       const cdfci_opts* opts, cdfci_ctx** out) {
  if (!dims || ndim < 1 || ndim > 3 || !out) return CDFCI_ERR_INVALID_ARG;
  int L = 1;
  for (int i = 0; i < ndim; ++i) {
    if (dims[i] < 1) return CDFCI_ERR_INVALID_ARG;
    L *= dims[i];
  }
  if (L > kMaxOrb) return CDFCI_ERR_UNSUPPORTED;
  int rc = make_ctx(L, n_alpha, n_beta, opts, out);
  if (rc) return rc;
  cdfci_ctx* c = *out;
  std::vector<double> h, eri;
  hubbard_integrals(dims, ndim, t, U, h, eri);
  rc = upload(c, h.data(), eri.data());
  uint64_t a0 = 0, b0 = 0;
  neel_determinant(dims, ndim, n_alpha, n_beta, &a0, &b0);
  int kind = c->opts.init_kind == 1 ? 1 : 2;
  if (!rc) rc = setup_and_init(c, kind, a0, b0);
  if (rc) {
    cdfci_free(c);
    *out = nullptr;
  }
  return rc;
}

static int run_cd1(cdfci_ctx* c, int64_t nsteps, double* trE, uint64_t* tra, uint64_t* trb,
                   double* treta, cdfci_stats* out) {
  if (!c) return CDFCI_ERR_INVALID_ARG;
  if (c->poisoned) return CDFCI_ERR_INVALID_ARG;
  if (nsteps < 0) return CDFCI_ERR_INVALID_ARG;
  Ctl before;
  int rc = ctl_read(c, &before);
  if (rc) return rc;
  if (before.sel_slot < 0 || (uint64_t)before.sel_slot >= c->nslots) return CDFCI_ERR_INVALID_ARG;
  double* dE = nullptr;
  uint64_t *da = nullptr, *db = nullptr;
  double* deta = nullptr;
  bool tracing = trE || tra || trb || treta;
  if (tracing) {
    // trace arrays are indexed by the global step, so offset by steps so far
    size_t n = (size_t)(before.steps + nsteps);
    HIP_TRY(hipMalloc(&dE, n * sizeof(double)));
    HIP_TRY(hipMalloc(&da, n * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&db, n * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&deta, n * sizeof(double)));
  }
  Cd1Args A;
  A.H = ham_of(c);
  A.T = c->T;
  A.mask = c->mask;
  A.max_entries = c->max_entries;
  A.ctl = c->ctl;
  A.parts = c->parts;
  A.nsteps = nsteps;
  A.n_col = c->n_col;
  A.tau = c->opts.z_threshold;
  A.theta = c->opts.dx_damping;
  A.dx_tol = c->opts.dx_threshold;
  A.tr_E = dE;
  A.tr_a = da;
  A.tr_b = db;
  A.tr_eta = deta;
  hipStream_t s = c->stream;
  k_reset_barrier<<<1, 1, 0, s>>>(c->ctl);
  HIP_TRY(hipEventRecord(c->ev0, s));
  if (nsteps > 0) {
    void* args[] = {&A};
    HIP_TRY(hipLaunchCooperativeKernel((const void*)k_cd1, dim3(c->grid), dim3(c->block), args, 0, s));
  }
  HIP_TRY(hipEventRecord(c->ev1, s));
  k_finish_steps<<<1, 1, 0, s>>>(c->ctl);
  HIP_TRY(hipGetLastError());
  Ctl h;
  rc = ctl_read(c, &h);
  if (rc) return rc;
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (tracing) {
    int64_t done = h.steps - before.steps;
    if (trE) {
      HIP_TRY(hipMemcpy(trE, dE + before.steps, done * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < done; ++i) trE[i] += c->shift;
    }
    if (tra) HIP_TRY(hipMemcpy(tra, da + before.steps, done * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (trb) HIP_TRY(hipMemcpy(trb, db + before.steps, done * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (treta) HIP_TRY(hipMemcpy(treta, deta + before.steps, done * sizeof(double), hipMemcpyDeviceToHost));
    (void)hipFree(dE);
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(deta);
  }
  if (out) {
    out->steps = h.steps - before.steps;
    out->total_steps = h.steps;
    out->elements = out->steps * c->n_col;
    out->inserts = (int64_t)(h.inserts - before.inserts);
    out->probes = 0;
    out->atomics = 0;
    out->occupied = h.occupied;
    out->max_probe = h.max_probe;
    out->stopped = h.stopped;
    out->energy = h.energy + c->shift;
    out->dx = h.d;
    out->mu = h.mu_hi + h.mu_lo;
    out->alpha = h.al_hi + h.al_lo;
    out->seconds = ms * 1e-3;
  }
  return check_error(c, h);
}

// ---- multicoordinate descent (Alg. 2) host orchestration

static constexpr int kMaxK = 1024;

// (Re)allocates the multicoordinate buffers.  A reallocation discards the
// candidate list, so *lost is set and the caller must rebuild it.
static int mc_alloc(cdfci_ctx* c, int k, uint64_t occupied, bool* lost) {
  *lost = false;
  // pages: one per scatter workgroup (k columns x chunks) plus the chosen set;
  // when the list is (re)built from the table (entering the multicoordinate
  // state) also enough for every stored entry.  Growth keeps 1/4 headroom.
  const uint64_t chunks = (uint64_t)((c->n_col + kPage - 1) / kPage);
  uint64_t pages = (uint64_t)k * chunks + (k + kPage - 1) / kPage;
  if (c->mode != 1) pages = std::max<uint64_t>(pages, (occupied + 1 + kPage - 1) / kPage);
  const uint64_t need_cand = pages * kPage;
  if (k > c->mc_kcap || need_cand > c->cand_cap) {
    // release and reallocate at the larger size
    void* olds[] = {c->cand, c->cnt, c->pkey, c->gkey, c->dslot, c->hii, c->sel_slot, c->sel_a, c->sel_b,
                    c->eta, c->pstat, c->chat, c->rec};
    for (void* p : olds)
      if (p) (void)hipFree(p);
    const int kc = std::max(k, c->mc_kcap);
    const uint64_t cc = std::max(need_cand + need_cand / 4, c->cand_cap);
    HIP_TRY(hipMalloc(&c->cand, cc * sizeof(unsigned)));
    HIP_TRY(hipMalloc(&c->cnt, (cc / kPage) * sizeof(unsigned)));
    HIP_TRY(hipMalloc(&c->pkey, cc * sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&c->gkey, (cc + (uint64_t)kSelBlocks * kPage) * sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&c->dslot, (cc + (uint64_t)kSelBlocks * kPage) * sizeof(unsigned)));
    HIP_TRY(hipMalloc(&c->hii, (size_t)kc * kc * sizeof(double)));
    HIP_TRY(hipMalloc(&c->sel_slot, (size_t)kc * sizeof(int64_t)));
    HIP_TRY(hipMalloc(&c->sel_a, (size_t)kc * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&c->sel_b, (size_t)kc * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&c->eta, (size_t)kc * sizeof(double)));
    HIP_TRY(hipMalloc(&c->chat, (size_t)kc * sizeof(double)));
    HIP_TRY(hipMalloc(&c->rec, (size_t)kc * chunks * kPage * sizeof(ScatRec)));
    c->pstat_cap = (uint64_t)kc * chunks * 4;
    HIP_TRY(hipMalloc(&c->pstat, (c->pstat_cap + kc) * sizeof(PageStat)));  // page quarters, then column sums
    c->mc_kcap = kc;
    c->cand_cap = cc;
    *lost = true;
  }
  if (!c->mst) {
    HIP_TRY(hipMalloc(&c->mst, sizeof(McState)));
    McState z;
    memset(&z, 0, sizeof(z));
    z.scale = 1.0;
    z.inv_scale = 1.0;
    z.pred_d = -1;
    HIP_TRY(hipMemcpyAsync(c->mst, &z, sizeof(z), hipMemcpyHostToDevice, c->stream));
    // two histograms: the selection's, and the second digits of k_mc_keys
    HIP_TRY(hipMalloc(&c->hist, 2 * kRadixBins * sizeof(unsigned)));
    HIP_TRY(hipMemsetAsync(c->hist, 0, 2 * kRadixBins * sizeof(unsigned), c->stream));
    HIP_TRY(hipMalloc(&c->dcount, kSelBlocks * sizeof(unsigned)));
    HIP_TRY(hipMalloc(&c->ties, kMaxTies * sizeof(unsigned)));
    c->bm_words = (c->nslots / 32 + 1 + 3) & ~3ull;  // whole 16-byte vectors
    HIP_TRY(hipMalloc(&c->bitmap, c->bm_words * sizeof(unsigned)));
  }
  return 0;
}

// single-coordinate state -> multicoordinate state: every stored entry is a
// candidate of the first multicoordinate selection (after init these are the
// columns of the starting determinants, as Alg. 2 prescribes)
static int enter_multi(cdfci_ctx* c) {
  hipStream_t s = c->stream;
  k_mc_clear<<<1024, 256, 0, s>>>(c->bitmap, c->bm_words, c->mst);
  k_mc_init_cands<<<2048, 256, 0, s>>>(c->T, c->nslots, c->cand, c->mst, c->cand_cap);
  k_mc_dense_pages<<<256, 256, 0, s>>>(c->cnt, c->mst, c->cand_cap);
  HIP_TRY(hipGetLastError());
  c->mode = 1;
  return 0;
}

// multicoordinate state -> single-coordinate state: fold the lazy scale into
// the table and choose the next coordinate over every stored entry
static int enter_single(cdfci_ctx* c) {
  hipStream_t s = c->stream;
  k_mc_rescale<<<2048, 256, 0, s>>>(c->T, c->nslots, c->mst, 1);
  k_mc_rescale_done<<<1, 1, 0, s>>>(c->mst, 1);
  int sel_blocks = (int)std::min<uint64_t>((c->nslots + 255) / 256, (uint64_t)c->max_parts);
  k_select_table<<<sel_blocks, 256, 0, s>>>(c->T, c->nslots, c->ctl, c->parts);
  k_select_final<<<1, 1, 0, s>>>(c->parts, sel_blocks, c->ctl);
  HIP_TRY(hipGetLastError());
  c->mode = 0;
  return 0;
}

static int run_mc(cdfci_ctx* c, int k, int64_t nsteps, double* trE, cdfci_stats* out) {
  if (c->poisoned) return CDFCI_ERR_INVALID_ARG;
  if (k > kMaxK || nsteps < 0) return CDFCI_ERR_INVALID_ARG;
  if (c->nslots > (1ull << 31)) return CDFCI_ERR_UNSUPPORTED;  // slot ids are 32-bit below an all-ones mark
  Ctl before;
  int rc = ctl_read(c, &before);
  if (rc) return rc;
  bool lost = false;
  rc = mc_alloc(c, k, before.occupied, &lost);
  if (rc) return rc;
  if (c->mode != 1 || lost) {
    rc = enter_multi(c);
    if (rc) return rc;
  }
  double* dE = nullptr;
  if (trE) HIP_TRY(hipMalloc(&dE, (size_t)(before.steps + nsteps + 1) * sizeof(double)));
  hipStream_t s = c->stream;
  const Ham H = ham_of(c);
  const int chunks = (int)((c->n_col + kPage - 1) / kPage);
  EigArgs ea{c->T, c->T, c->sel_slot, c->hii, c->mst, c->ctl, c->eta, c->chat, k,
             c->opts.dx_damping, c->opts.dx_threshold, dE,
             ProbeArgs{H, c->mask, c->sel_a, c->sel_b, c->cand, c->pstat, c->rec, c->n_col}, nullptr};
  ApplyArgs aa{H,      c->T,    c->mask,  c->sel_a, c->sel_b,           c->eta, c->mst, c->pstat,
               c->rec, c->cand, c->n_col, c->opts.z_threshold, k};
  const unsigned page0 = (unsigned)(k * chunks);
  k_reset_barrier<<<1, 1, 0, s>>>(c->ctl);
  if (c->timing)
    while ((int64_t)c->tev.size() < 6 * nsteps) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      c->tev.push_back(e);
    }
  auto mark = [&](int64_t step, int q) {
    return c->timing ? hipEventRecord(c->tev[(size_t)(6 * step + q)], s) : hipSuccess;
  };
  if (c->timing && nsteps > 0) {
    if (c->ptime_cap < nsteps) {
      if (c->ptime) (void)hipFree(c->ptime);
      c->ptime = nullptr;
      HIP_TRY(hipMalloc(&c->ptime, (size_t)4 * nsteps * sizeof(unsigned long long)));
      c->ptime_cap = nsteps;
    }
    k_ptime_init<<<(unsigned)std::min<int64_t>((nsteps + 255) / 256, 1024), 256, 0, s>>>(c->ptime, nsteps);
  }
  // one step's launches on stream q, with the phase events when timing
  auto launch_step = [&](hipStream_t q, int64_t step) -> hipError_t {
    hipError_t e = hipSuccess;
    auto mk = [&](int which) {
      if (e == hipSuccess) e = mark(step, which);
    };
    mk(0);
    ea.ptime = c->timing ? c->ptime + 4 * step : nullptr;
    // keys of every position, the bound the repeats allow, the exact pass
    // (repeats dropped) over the keys above it, and the rest of the
    // selection: one workgroup for k <= kTailMaxK, else the digit of pass 0
    // in one workgroup and grid passes
    const SelBufs sb{c->gkey, c->dslot, c->dcount};
    k_mc_keys<<<kSelBlocks, 256, 0, q>>>(c->T, c->cand, c->cnt, c->pkey, c->ctl, c->mst, c->hist,
                                         c->hist + kRadixBins);
    k_mc_bound<<<1, 256, 0, q>>>(c->mst, c->ctl, c->hist, c->hist + kRadixBins, k);
    k_mc_dedup<<<kSelBlocks, 256, 0, q>>>(c->cand, c->pkey, sb, c->mst, c->hist, c->bitmap);
    if (k <= kTailMaxK) {
      k_mc_tail<<<1, kTailThreads, 0, q>>>(c->T, sb, c->mst, c->ctl, c->hist, c->sel_slot, c->sel_a, c->sel_b,
                                           k, c->bitmap, 1);
    } else {
      k_mc_tail<<<1, kTailThreads, 0, q>>>(c->T, sb, c->mst, c->ctl, c->hist, c->sel_slot, c->sel_a, c->sel_b,
                                           k, c->bitmap, 0);
      for (int pass = 1; pass < kRadixPasses; ++pass)
        k_mc_radix<<<kSelBlocks, 256, 0, q>>>(c->T, c->cand, c->cnt, sb, c->ctl, c->mst, c->hist, pass, 0, k);
      k_mc_gather_ties<<<kSelBlocks, 256, 0, q>>>(c->T, sb, c->mst, c->sel_slot, c->ties, c->sel_a, c->sel_b, k,
                                                  c->bitmap);
    }
    mk(1);
    k_mc_hii<<<k, 256, 0, q>>>(H, c->sel_a, c->sel_b, c->mst, c->hii, k, c->cnt, c->n_col);
    mk(2);
    // workgroup 0 solves the reduced problem; the others run the probe half
    // of the scatter
    if (k <= kEigSmall)
      k_mc_lobpcg<kEigSmall, 512><<<kEigGridSmall, 512, 0, q>>>(ea);
    else if (k <= 256)
      k_mc_lobpcg<256, 1024><<<kEigGrid, 1024, 0, q>>>(ea);
    else
      k_mc_lobpcg<kMaxK, 1024><<<kEigGrid, 1024, 0, q>>>(ea);
    mk(3);
    k_mc_apply<<<dim3(chunks, k), 256, 0, q>>>(aa);
    mk(4);
    k_mc_colfinish<<<k, 256, 0, q>>>(c->pstat, chunks, c->pstat + c->pstat_cap, c->hii, c->chat, c->T,
                                     c->sel_slot, c->cand, c->cnt, c->mst, c->ctl, c->max_entries, page0, k);
    k_mc_rescale<<<256, 256, 0, q>>>(c->T, c->nslots, c->mst, 0);
    mk(5);
    return e;
  };
  HIP_TRY(hipEventRecord(c->ev0, s));
  for (int64_t step = 0; step < nsteps; ++step) {
    HIP_TRY(launch_step(s, step));
    if (((step + 1) & 63) == 0) HIP_TRY(hipGetLastError());
  }
  k_mc_rescale_done<<<1, 1, 0, s>>>(c->mst, 0);  // inside the loop k_mc_bound does this
  HIP_TRY(hipEventRecord(c->ev1, s));
  HIP_TRY(hipGetLastError());
  Ctl h;
  rc = ctl_read(c, &h);
  if (rc) return rc;
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  const int64_t done = h.steps - before.steps;
  if (c->timing && nsteps > 0) {
    std::vector<unsigned long long> pt((size_t)4 * nsteps);
    HIP_TRY(hipMemcpy(pt.data(), c->ptime, pt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    for (int64_t step = 0; step < nsteps; ++step) {
      for (int q = 0; q < 5; ++q) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, c->tev[(size_t)(6 * step + q)], c->tev[(size_t)(6 * step + q + 1)]));
        c->t_phase_mc[q] += 1e-3 * t;
      }
      const unsigned long long t0 = pt[(size_t)(4 * step)], t1 = pt[(size_t)(4 * step + 1)];
      if (t0 != ~0ull && t1 > t0 && khz > 0) c->t_phase_mc[5] += (double)(t1 - t0) / (1e3 * khz);
      const unsigned long long t2 = pt[(size_t)(4 * step + 2)], t3 = pt[(size_t)(4 * step + 3)];
      if (t3 > t2 && t2 > 0 && khz > 0) c->t_phase_mc[6] += (double)(t3 - t2) / (1e3 * khz);
      ++c->n_timed;
    }
  }
  if (trE) {
    if (done > 0) HIP_TRY(hipMemcpy(trE, dE + before.steps, done * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < done; ++i) trE[i] += c->shift;
    (void)hipFree(dE);
  }
  if (out) {
    out->steps = done;
    out->total_steps = h.steps;
    out->elements = done * (int64_t)k * c->n_col;
    out->inserts = (int64_t)(h.inserts - before.inserts);
    out->probes = (int64_t)(h.probes - before.probes);
    out->atomics = (int64_t)(h.atomics - before.atomics);
    out->occupied = h.occupied;
    out->max_probe = h.max_probe;
    out->stopped = h.stopped;
    out->energy = h.energy + c->shift;
    out->dx = h.d;
    out->mu = h.mu_hi + h.mu_lo;
    out->alpha = h.al_hi + h.al_lo;
    out->seconds = ms * 1e-3;
  }
  return check_error(c, h);
}

int cdfci_step(cdfci_ctx* ctx, int k, int64_t nsteps, cdfci_stats* out) {
  if (!ctx || k < 1) return CDFCI_ERR_INVALID_ARG;
  if (k == 1) {
    if (ctx->mode == 1) {
      int rc = enter_single(ctx);
      if (rc) return rc;
    }
    return run_cd1(ctx, nsteps, nullptr, nullptr, nullptr, nullptr, out);
  }
  return run_mc(ctx, k, nsteps, nullptr, out);
}

int cdfci_step_energies(cdfci_ctx* ctx, int k, int64_t nsteps, double* energy, cdfci_stats* out) {
  if (!ctx || k < 1 || !energy) return CDFCI_ERR_INVALID_ARG;
  if (k == 1) {
    if (ctx->mode == 1) {
      int rc = enter_single(ctx);
      if (rc) return rc;
    }
    return run_cd1(ctx, nsteps, energy, nullptr, nullptr, nullptr, out);
  }
  return run_mc(ctx, k, nsteps, energy, out);
}

int cdfci_step_trace(cdfci_ctx* ctx, int64_t nsteps, double* energy, uint64_t* sel_alpha,
                     uint64_t* sel_beta, double* eta, cdfci_stats* out) {
  if (!ctx) return CDFCI_ERR_INVALID_ARG;
  if (ctx->mode == 1) {
    int rc = enter_single(ctx);
    if (rc) return rc;
  }
  return run_cd1(ctx, nsteps, energy, sel_alpha, sel_beta, eta, out);
}

int cdfci_energy(cdfci_ctx* c, int exact, double* energy) {
  if (!c || !energy) return CDFCI_ERR_INVALID_ARG;
  Ctl h;
  int rc = ctl_read(c, &h);
  if (rc) return rc;
  if (!exact) {
    *energy = (h.al_hi + h.al_lo) / (h.mu_hi + h.mu_lo) + c->shift;
    return 0;
  }
  hipStream_t s = c->stream;
  unsigned long long* d_cnt = (unsigned long long*)(c->dscratch + 2 * 4096 + 4);
  HIP_TRY(hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long), s));
  rc = ensure_list(c, (int64_t)h.occupied + 1);
  if (rc) return rc;
  k_compact<<<2048, 256, 0, s>>>(c->T, c->nslots, 1, c->list, d_cnt, c->list_cap);
  unsigned long long n = 0;
  HIP_TRY(hipMemcpyAsync(&n, d_cnt, sizeof(n), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((int64_t)n > c->list_cap) return CDFCI_ERR_INVALID_ARG;
  int nb = 2048;
  k_apply_energy<<<nb, 256, 0, s>>>(ham_of(c), c->T, c->mask, c->list, (int64_t)n, c->n_col,
                                    c->dscratch, c->dscratch + 4096);
  k_sum_partials<<<1, 1, 0, s>>>(c->dscratch, c->dscratch + 4096, nb, c->dscratch + 2 * 4096);
  HIP_TRY(hipGetLastError());
  double r[2];
  HIP_TRY(hipMemcpyAsync(r, c->dscratch + 2 * 4096, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *energy = r[0] / r[1] + c->shift;
  return 0;
}

int cdfci_rdm_backward(cdfci_ctx* c, double grad_E, int64_t top_n, double* energy, double* dh,
                       double* deri, double* kappa) {
  if (!c) return CDFCI_ERR_INVALID_ARG;
  CallBufs bufs;
  int64_t* sel = nullptr;
  int64_t n = 0;
  int rc = select_support(c, top_n, bufs, &sel, &n);
  if (rc) return rc;
  hipStream_t s = c->stream;
  const int N = c->N;
  const size_t N2 = (size_t)N * N, N4 = N2 * N2;
  const Ham H = ham_of(c);
  // normalisation and the support table (load <= 1/2)
  double* part;
  HIP_TRY(bufs.alloc(&part, 2 * 1024 + 8));
  k_rdm_norm<<<1024, 256, 0, s>>>(c->T, sel, n, part);
  k_sum_partials<<<1, 1, 0, s>>>(part, part, 1024, part + 2048);
  uint64_t ss = 1024;
  while (ss < 2 * (uint64_t)n) ss <<= 1;
  Slot* S;
  uint64_t *sa, *sb;
  double *sc, *Y1, *Z, *g1, *g2, *F2, *dkap, *ddh;
  int* err;
  HIP_TRY(bufs.alloc(&S, ss));
  HIP_TRY(bufs.alloc(&sa, n));
  HIP_TRY(bufs.alloc(&sb, n));
  HIP_TRY(bufs.alloc(&sc, n));
  HIP_TRY(bufs.alloc(&err, 1));
  HIP_TRY(bufs.alloc(&Y1, N2));
  HIP_TRY(bufs.alloc(&Z, N4));
  HIP_TRY(bufs.alloc(&g1, N2));
  HIP_TRY(bufs.alloc(&g2, N4));
  HIP_TRY(bufs.alloc(&F2, N2));
  HIP_TRY(bufs.alloc(&dkap, N2));
  HIP_TRY(bufs.alloc(&ddh, N2));
  HIP_TRY(hipMemsetAsync(err, 0, sizeof(int), s));
  HIP_TRY(hipMemsetAsync(Y1, 0, N2 * sizeof(double), s));
  HIP_TRY(hipMemsetAsync(Z, 0, N4 * sizeof(double), s));
  HIP_TRY(hipMemsetAsync(F2, 0, N2 * sizeof(double), s));
  double* e_acc = part + 2048 + 2;  // direct c^T H c of the normalised support
  HIP_TRY(hipMemsetAsync(e_acc, 0, sizeof(double), s));
  k_clear_table<<<1024, 256, 0, s>>>(S, ss);
  k_rdm_build<<<1024, 256, 0, s>>>(c->T, sel, n, part + 2048, S, ss - 1, sa, sb, sc, err);
  // pair and diagonal contributions
  k_rdm_pairs<<<(int)std::min<int64_t>(n, 16384), 256, 0, s>>>(H, S, ss - 1, sa, sb, sc, n, c->n_col, Y1,
                                                                Z, e_acc);
  k_rdm_symmetrize<<<2048, 256, 0, s>>>(Y1, Z, N, g1, g2);
  const size_t shm = (size_t)(N + 2 * N * N) * sizeof(double);
  k_rdm_diag<<<(int)std::min<int64_t>(n, 512), 256, shm, s>>>(H, sa, sb, sc, n, g1, g2, e_acc);
  // kappa: F2 on the FP64 matrix cores, then F, kappa and dh
  const int tiles = (N + 15) / 16;
  const int slices = (int)(((int64_t)N * N * N + kKappaSlice - 1) / kKappaSlice);
  k_kappa_mfma<<<dim3(tiles * tiles, slices), 64, 0, s>>>(c->d_eri, g2, N, F2);
  k_kappa_finish<<<(int)((N2 + 255) / 256), 256, 0, s>>>(c->d_h, g1, F2, N, grad_E, dkap, ddh);
  // energy from the RDMs; g2 becomes deri
  k_rdm_outputs<<<1024, 256, 0, s>>>(c->d_h, c->d_eri, g1, g2, N, grad_E, part + 1024);
  k_sum_partials<<<1, 1, 0, s>>>(part + 1024, part + 1024, 1024, part + 2048 + 4);
  HIP_TRY(hipGetLastError());
  int herr = 0;
  double he[8];
  HIP_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(he, part + 2048, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (dh) HIP_TRY(hipMemcpyAsync(dh, ddh, N2 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (kappa) HIP_TRY(hipMemcpyAsync(kappa, dkap, N2 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (deri) HIP_TRY(hipMemcpyAsync(deri, g2, N4 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (herr) return CDFCI_ERR_TABLE_FULL;
  if (energy) {
    energy[0] = he[4] + c->shift;
    energy[1] = he[2] + c->shift;
  }
  return 0;
}

int cdfci_column(cdfci_ctx* c, const uint64_t key[2], uint64_t* keys, double* vals, int64_t cap,
                 int64_t* count) {
  if (!c || !key || !count) return CDFCI_ERR_INVALID_ARG;
  if (__builtin_popcountll(key[0]) != c->na || __builtin_popcountll(key[1]) != c->nb ||
      (c->N < 64 && ((key[0] | key[1]) >> c->N)))
    return CDFCI_ERR_INVALID_ARG;
  *count = c->n_col;
  if (cap < c->n_col || !keys || !vals) return CDFCI_ERR_INVALID_ARG;
  uint64_t* dk;
  double* dv;
  HIP_TRY(hipMalloc(&dk, 2 * c->n_col * sizeof(uint64_t)));
  HIP_TRY(hipMalloc(&dv, c->n_col * sizeof(double)));
  int blocks = (int)std::min<int64_t>((c->n_col + 255) / 256, 4096);
  k_column<<<blocks, 256, 0, c->stream>>>(ham_of(c), key[0], key[1], c->n_col, c->shift, dk, dv);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(keys, dk, 2 * c->n_col * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(vals, dv, c->n_col * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  (void)hipFree(dk);
  (void)hipFree(dv);
  return 0;
}

int cdfci_column_noalloc(cdfci_ctx* c, const uint64_t key[2], uint64_t* keys, double* vals, int64_t cap,
                         int64_t* count) {
  if (!c || !key || !count) return CDFCI_ERR_INVALID_ARG;
  if (__builtin_popcountll(key[0]) != c->na || __builtin_popcountll(key[1]) != c->nb ||
      (c->N < 64 && ((key[0] | key[1]) >> c->N)))
    return CDFCI_ERR_INVALID_ARG;
  *count = c->n_col;
  if (c->n_col > kNoAllocMaxEntries) return CDFCI_ERR_UNSUPPORTED;
  if (cap < c->n_col || !keys || !vals) return CDFCI_ERR_INVALID_ARG;
  if (c->device < 0 || c->device >= kMaxDevices || !g_scratch_ptr[c->device]) return CDFCI_ERR_HIP;
  // the staging buffer is this device's copy of `scratch`, by the address
  // resolved at set-up (never the host-side name of the array)
  unsigned char* base = (unsigned char*)g_scratch_ptr[c->device];
  uint64_t* dk = (uint64_t*)base;
  double* dv = (double*)(base + kNoAllocMaxEntries * 2 * sizeof(uint64_t));
  int blocks = (int)std::min<int64_t>((c->n_col + 255) / 256, 4096);
  k_column<<<blocks, 256, 0, c->stream>>>(ham_of(c), key[0], key[1], c->n_col, c->shift, dk, dv);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(keys, dk, 2 * c->n_col * sizeof(uint64_t), hipMemcpyDefault, c->stream));
  HIP_TRY(hipMemcpyAsync(vals, dv, c->n_col * sizeof(double), hipMemcpyDefault, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return 0;
}

int cdfci_entry(cdfci_ctx* c, const uint64_t k1[2], const uint64_t k2[2], double* value) {
  if (!c || !k1 || !k2 || !value) return CDFCI_ERR_INVALID_ARG;
  double* d;
  HIP_TRY(hipMalloc(&d, sizeof(double)));
  k_entry<<<1, 1, 0, c->stream>>>(ham_of(c), k1[0], k1[1], k2[0], k2[1], d);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(value, d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  (void)hipFree(d);
  if (k1[0] == k2[0] && k1[1] == k2[1]) *value += c->shift;  // entries of H
  return 0;
}

int cdfci_export(cdfci_ctx* c, int64_t top_n, uint64_t* keys, double* cv, double* bv, int64_t cap,
                 int64_t* count) {
  if (!c || !count) return CDFCI_ERR_INVALID_ARG;
  hipStream_t s = c->stream;
  if (top_n > 0) {
    CallBufs bufs;
    int64_t* sel = nullptr;
    int64_t n = 0;
    int rc = select_support(c, top_n, bufs, &sel, &n);
    if (rc) return rc;
    *count = n;
    const int64_t m = std::min(n, cap);
    if (m > 0 && keys && cv && bv) {
      uint64_t* dk;
      double *dc, *db;
      HIP_TRY(bufs.alloc(&dk, 2 * m));
      HIP_TRY(bufs.alloc(&dc, m));
      HIP_TRY(bufs.alloc(&db, m));
      k_gather<<<1024, 256, 0, s>>>(c->T, sel, m, dk, dc, db);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(keys, dk, 2 * m * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(cv, dc, m * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(bv, db, m * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return 0;
  }
  if (c->mode == 1) {  // true values: fold the multicoordinate lazy scale in
    k_mc_rescale<<<2048, 256, 0, s>>>(c->T, c->nslots, c->mst, 1);
    k_mc_rescale_done<<<1, 1, 0, s>>>(c->mst, 1);
  }
  Ctl h;
  int rc = ctl_read(c, &h);
  if (rc) return rc;
  unsigned long long* d_cnt = (unsigned long long*)(c->dscratch + 2 * 4096 + 4);
  HIP_TRY(hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long), s));
  rc = ensure_list(c, (int64_t)h.occupied + 1);
  if (rc) return rc;
  k_compact<<<2048, 256, 0, s>>>(c->T, c->nslots, 0, c->list, d_cnt, c->list_cap);
  unsigned long long n = 0;
  HIP_TRY(hipMemcpyAsync(&n, d_cnt, sizeof(n), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *count = (int64_t)n;
  int64_t m = std::min<int64_t>(std::min<int64_t>((int64_t)n, cap), c->list_cap);
  if (m > 0 && keys && cv && bv) {
    uint64_t* dk;
    double *dc, *db;
    HIP_TRY(hipMalloc(&dk, 2 * m * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&dc, m * sizeof(double)));
    HIP_TRY(hipMalloc(&db, m * sizeof(double)));
    k_gather<<<1024, 256, 0, s>>>(c->T, c->list, m, dk, dc, db);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(keys, dk, 2 * m * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(cv, dc, m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(bv, db, m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipFree(dk);
    (void)hipFree(dc);
    (void)hipFree(db);
  }
  return 0;
}

int cdfci_mc_candidates(cdfci_ctx* c, uint64_t* keys, double* g, double* cv, double* bv, int64_t cap,
                        int64_t* count, double* mu_scale) {
  if (!c || !count || cap < 0) return CDFCI_ERR_INVALID_ARG;
  if (c->mode != 1 || !c->mst) return CDFCI_ERR_INVALID_ARG;
  hipStream_t s = c->stream;
  McState st;
  HIP_TRY(hipMemcpyAsync(&st, c->mst, sizeof(st), hipMemcpyDeviceToHost, s));
  Ctl h;
  int rc = ctl_read(c, &h);
  if (rc) return rc;
  CallBufs bufs;
  const uint64_t m = std::max<uint64_t>((uint64_t)cap, 1);
  uint64_t* dk;
  double *dg, *dc, *db;
  unsigned long long* dn;
  HIP_TRY(bufs.alloc(&dk, 2 * m));
  HIP_TRY(bufs.alloc(&dg, m));
  HIP_TRY(bufs.alloc(&dc, m));
  HIP_TRY(bufs.alloc(&db, m));
  HIP_TRY(bufs.alloc(&dn, 1));
  HIP_TRY(hipMemsetAsync(dn, 0, sizeof(unsigned long long), s));
  k_mc_export_cands<<<1024, 256, 0, s>>>(c->T, c->cand, c->cnt, c->mst, c->ctl, dk, dg, dc, db,
                                         (unsigned long long)cap, dn, c->bitmap);
  k_mc_clear_words<<<1024, 256, 0, s>>>(c->bitmap, c->bm_words);  // clear again for the next selection
  HIP_TRY(hipGetLastError());
  unsigned long long n = 0;
  HIP_TRY(hipMemcpyAsync(&n, dn, sizeof(n), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *count = (int64_t)n;
  const int64_t w = std::min<int64_t>((int64_t)n, cap);
  if (w > 0) {
    if (keys) HIP_TRY(hipMemcpyAsync(keys, dk, 2 * w * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    if (g) HIP_TRY(hipMemcpyAsync(g, dg, w * sizeof(double), hipMemcpyDeviceToHost, s));
    if (cv) HIP_TRY(hipMemcpyAsync(cv, dc, w * sizeof(double), hipMemcpyDeviceToHost, s));
    if (bv) HIP_TRY(hipMemcpyAsync(bv, db, w * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (mu_scale) {
    mu_scale[0] = h.mu_hi + h.mu_lo;
    mu_scale[1] = st.scale;
  }
  return 0;
}

int cdfci_mc_selection(cdfci_ctx* c, uint64_t* keys, double* eta, int64_t cap, int64_t* count) {
  if (!c || !count || cap < 0) return CDFCI_ERR_INVALID_ARG;
  if (!c->mst || !c->sel_a) return CDFCI_ERR_INVALID_ARG;
  hipStream_t s = c->stream;
  McState st;
  HIP_TRY(hipMemcpyAsync(&st, c->mst, sizeof(st), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t n = (int64_t)st.last_sel;
  *count = n;
  const int64_t w = std::min<int64_t>(n, cap);
  if (w > 0) {
    std::vector<uint64_t> a((size_t)w), b((size_t)w);
    HIP_TRY(hipMemcpyAsync(a.data(), c->sel_a, w * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(b.data(), c->sel_b, w * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    if (eta) HIP_TRY(hipMemcpyAsync(eta, c->eta, w * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (keys)
      for (int64_t i = 0; i < w; ++i) {
        keys[2 * i] = a[(size_t)i];
        keys[2 * i + 1] = b[(size_t)i];
      }
  }
  return 0;
}

int cdfci_random_access_rates(uint64_t table_slots, int64_t n_ops, double* rates) {
  if (!rates || n_ops < 1 || table_slots < 1024 || (table_slots & (table_slots - 1))) return CDFCI_ERR_INVALID_ARG;
  CallBufs bufs;
  Slot* T;
  unsigned* bm;
  unsigned long long* sink;
  const uint64_t ncopy = (1ull << 30) / sizeof(double4);
  double4 *ca, *cb;
  HIP_TRY(bufs.alloc(&T, table_slots));
  HIP_TRY(bufs.alloc(&bm, table_slots / 32));
  HIP_TRY(bufs.alloc(&sink, 1));
  HIP_TRY(bufs.alloc(&ca, ncopy));
  HIP_TRY(bufs.alloc(&cb, ncopy));
  HIP_TRY(hipMemset(bm, 0, table_slots / 32 * sizeof(unsigned)));
  HIP_TRY(hipMemset(ca, 0, ncopy * sizeof(double4)));
  k_ra_fill<<<4096, 256>>>(T, table_slots);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int grid = (int)((n_ops + 255) / 256);
  int rc = 0;
  for (int kind = 0; kind < 5 && !rc; ++kind) {
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      if (hipEventRecord(e0) != hipSuccess) rc = CDFCI_ERR_HIP;
      if (kind < 4)
        k_ra<<<grid, 256>>>(T, bm, table_slots - 1, (uint64_t)n_ops, 1000003ull * (rep + 1) + kind, kind, sink);
      else
        k_ra_copy<<<4096, 256>>>(ca, cb, ncopy);
      if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) rc = CDFCI_ERR_HIP;
      float ms = 0.0f;
      if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = CDFCI_ERR_HIP;
      if (rep > 0 && ms < best) best = ms;  // the first run warms up
    }
    rates[kind] = kind < 4 ? (double)n_ops / (best * 1e-3) : 2.0 * (double)(1ull << 30) / (best * 1e-3);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!rc && hipGetLastError() != hipSuccess) rc = CDFCI_ERR_HIP;
  return rc;
}

int cdfci_load(cdfci_ctx* c, const uint64_t* keys, const double* cv, int64_t count) {
  if (!c || !keys || !cv || count < 1) return CDFCI_ERR_INVALID_ARG;
  if ((uint64_t)count > c->max_entries) return CDFCI_ERR_TABLE_FULL;
  const uint64_t valid = c->N == 64 ? ~0ull : ((1ull << c->N) - 1);
  std::vector<InitTask> tasks((size_t)count);
  bool any = false;
  for (int64_t i = 0; i < count; ++i) {
    const uint64_t a = keys[2 * i], b = keys[2 * i + 1];
    if ((a & ~valid) || (b & ~valid) || __builtin_popcountll(a) != c->na || __builtin_popcountll(b) != c->nb ||
        !std::isfinite(cv[i]))
      return CDFCI_ERR_INVALID_ARG;
    any = any || cv[i] != 0.0;
    tasks[i] = InitTask{a, b, cv[i]};
  }
  if (!any) return CDFCI_ERR_INVALID_ARG;
  hipStream_t s = c->stream;
  if (c->mode == 1) {  // the multicoordinate scale no longer applies
    k_mc_rescale_done<<<1, 1, 0, s>>>(c->mst, 1);
    c->mode = 0;
  }
  CallBufs bufs;
  InitTask* d_tasks;
  unsigned long long* d_dup;
  HIP_TRY(bufs.alloc(&d_tasks, (uint64_t)count));
  HIP_TRY(bufs.alloc(&d_dup, 1));
  HIP_TRY(hipMemcpyAsync(d_tasks, tasks.data(), count * sizeof(InitTask), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(d_dup, 0, sizeof(unsigned long long), s));
  k_zero_ctl<<<1, 1, 0, s>>>(c->ctl);
  k_clear_table<<<2048, 256, 0, s>>>(c->T, c->nslots);
  k_load_insert<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(c->T, c->mask, d_tasks, count, c->ctl, d_dup);
  // one workgroup per (column chunk, determinant), at most 65535 determinants a launch
  const Ham H = ham_of(c);
  const int chunks = (int)std::min<int64_t>((c->n_col + 255) / 256, count > 4096 ? 8 : 256);
  for (int pass = 0; pass < 2; ++pass)
    for (int64_t off = 0; off < count; off += 65535) {
      const int nb = (int)std::min<int64_t>(65535, count - off);
      k_load_scatter<<<dim3(chunks, nb), 256, 0, s>>>(H, c->T, c->mask, d_tasks + off, c->n_col, c->ctl,
                                                      c->opts.z_threshold, pass);
    }
  const int sb = 1024;
  k_table_scalars<<<sb, 256, 0, s>>>(c->T, c->nslots, c->dscratch);
  k_table_scalars_final<<<1, 1, 0, s>>>(c->dscratch, sb, c->ctl);
  const int sel_blocks = (int)std::min<uint64_t>((c->nslots + 255) / 256, (uint64_t)c->max_parts);
  k_select_table<<<sel_blocks, 256, 0, s>>>(c->T, c->nslots, c->ctl, c->parts);
  k_select_final<<<1, 1, 0, s>>>(c->parts, sel_blocks, c->ctl);
  HIP_TRY(hipGetLastError());
  unsigned long long dup = 0;
  HIP_TRY(hipMemcpyAsync(&dup, d_dup, sizeof(dup), hipMemcpyDeviceToHost, s));
  Ctl h;
  int rc = ctl_read(c, &h);
  if (rc) return rc;
  c->poisoned = false;
  rc = check_error(c, h);
  if (rc) return rc;
  if (dup) {
    c->poisoned = true;
    return CDFCI_ERR_INVALID_ARG;
  }
  return 0;
}

int cdfci_set_threshold(cdfci_ctx* c, double tau) {
  if (!c || !(tau >= 0.0) || !std::isfinite(tau)) return CDFCI_ERR_INVALID_ARG;
  c->opts.z_threshold = tau;
  return 0;
}

int cdfci_step_search(cdfci_ctx* c, int64_t nsteps, int64_t chunk, double fill, double growth, double tau0,
                      double* tau_out, cdfci_stats* out) {
  if (!c || nsteps < 0 || chunk < 1 || !(fill > 0.0 && fill <= 1.0) || !(growth > 1.0) || !(tau0 > 0.0))
    return CDFCI_ERR_INVALID_ARG;
  cdfci_stats acc;
  memset(&acc, 0, sizeof(acc));
  double seconds = 0.0;
  int64_t done = 0, elements = 0, inserts = 0;
  int rc = 0;
  const double limit = fill * (double)c->max_entries;
  // one iteration stores at most a column's worth of new entries, so a chunk
  // started below the budget cannot pass the table's own limit
  const int64_t safe = std::max<int64_t>(1, (int64_t)(((double)c->max_entries - limit) / (double)c->n_col));
  chunk = std::min(chunk, safe);
  while (done < nsteps) {
    cdfci_stats st;
    rc = cdfci_step(c, 1, std::min(chunk, nsteps - done), &st);
    if (rc) return rc;
    done += st.steps;
    seconds += st.seconds;
    elements += st.elements;
    inserts += st.inserts;
    acc = st;
    if (st.stopped || st.steps == 0) break;
    if ((double)st.occupied <= limit) continue;
    // over budget: keep the support, raise tau, rebuild b on the smaller set
    int64_t n = 0;
    rc = cdfci_export(c, 0, nullptr, nullptr, nullptr, 0, &n);
    if (rc) return rc;
    std::vector<uint64_t> keys(2 * (size_t)n);
    std::vector<double> cv((size_t)n), bv((size_t)n);
    rc = cdfci_export(c, 0, keys.data(), cv.data(), bv.data(), n, &n);
    if (rc) return rc;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
      if (cv[i] != 0.0) {
        keys[2 * m] = keys[2 * i];
        keys[2 * m + 1] = keys[2 * i + 1];
        cv[m++] = cv[i];
      }
    for (;;) {
      c->opts.z_threshold = c->opts.z_threshold > 0.0 ? c->opts.z_threshold * growth : tau0;
      rc = cdfci_load(c, keys.data(), cv.data(), m);
      if (rc && rc != CDFCI_ERR_TABLE_FULL) return rc;
      Ctl h;
      if (!rc) {
        rc = ctl_read(c, &h);
        if (rc) return rc;
        if ((double)h.occupied <= limit) break;
      }
      if (c->opts.z_threshold > 1e3) return CDFCI_ERR_TABLE_FULL;  // the support alone does not fit
    }
  }
  if (tau_out) *tau_out = c->opts.z_threshold;
  if (out) {
    *out = acc;
    out->steps = done;
    out->elements = elements;
    out->inserts = inserts;
    out->probes = 0;
    out->atomics = 0;
    out->seconds = seconds;
  }
  return 0;
}

int cdfci_free(cdfci_ctx* c) {
  if (!c) return 0;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->own_table && c->T) (void)hipFree(c->T);
  if (c->d_h) (void)hipFree(c->d_h);
  if (c->d_eri) (void)hipFree(c->d_eri);
  if (c->d_eri8) (void)hipFree(c->d_eri8);
  if (c->d_jk) (void)hipFree(c->d_jk);
  if (c->ctl) (void)hipFree(c->ctl);
  if (c->parts) (void)hipFree(c->parts);
  if (c->list) (void)hipFree(c->list);
  if (c->dscratch) (void)hipFree(c->dscratch);
  void* mc[] = {c->mst, c->cand, c->cnt, c->pkey, c->gkey, c->dslot, c->dcount, c->ptime, c->hist, c->ties, c->sel_slot, c->sel_a, c->sel_b,
                c->eta, c->pstat, c->hii, c->bitmap, c->chat, c->rec};
  for (void* p : mc)
    if (p) (void)hipFree(p);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  delete c;
  return 0;
}

// ---------------------------------------------------------------------------
// Batches of Hubbard lattices: a memory-budgeted scheduler over one
// persistent kernel.  Instances are created when first admitted; the tables
// of the resident ones stay within the budget.

// The wavefunction of a context (stored entries with c != 0, true scale) into
// host vectors: keys interleaved (alpha, beta) and c.  Device memory used:
// the context's slot list, sized to that support only.
static int export_support(cdfci_ctx* c, std::vector<uint64_t>& keys, std::vector<double>& cv) {
  hipStream_t s = c->stream;
  if (c->mode == 1) {  // true values: fold the multicoordinate lazy scale in
    k_mc_rescale<<<2048, 256, 0, s>>>(c->T, c->nslots, c->mst, 1);
    k_mc_rescale_done<<<1, 1, 0, s>>>(c->mst, 1);
  }
  unsigned long long* d_cnt = (unsigned long long*)(c->dscratch + 2 * 4096 + 4);
  unsigned long long n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    HIP_TRY(hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long), s));
    k_compact<<<2048, 256, 0, s>>>(c->T, c->nslots, 1, c->list, d_cnt, c->list_cap);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&n, d_cnt, sizeof(n), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((int64_t)n <= c->list_cap) break;
    const int rc = ensure_list(c, (int64_t)n);
    if (rc) return rc;
  }
  keys.assign(2 * n, 0);
  cv.assign(n, 0.0);
  if (n == 0) return 0;
  CallBufs bufs;
  uint64_t* dk;
  double *dc, *db;
  HIP_TRY(bufs.alloc(&dk, 2 * n));
  HIP_TRY(bufs.alloc(&dc, n));
  HIP_TRY(bufs.alloc(&db, n));
  k_gather<<<1024, 256, 0, s>>>(c->T, c->list, (int64_t)n, dk, dc, db);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(keys.data(), dk, 2 * n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(cv.data(), dc, n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

static uint64_t batch_bytes(const cdfci_batch* B, int i) { return B->slots[i] * sizeof(Slot); }

// release instance i; its table goes to the pool (still counted as held)
static int batch_release(cdfci_batch* B, int i) {
  if (!B->ctx[i]) return 0;
  cdfci_free(B->ctx[i]);
  B->ctx[i] = nullptr;
  B->pool.push_back({batch_bytes(B, i), B->table_of[i]});
  B->table_of[i] = nullptr;
  return 0;
}

// a table buffer of `bytes` from the pool, or a new one; pooled buffers of
// other sizes are freed first when the budget would be exceeded
static int batch_table(cdfci_batch* B, uint64_t bytes, void** out) {
  for (size_t q = 0; q < B->pool.size(); ++q)
    if (B->pool[q].first == bytes) {
      *out = B->pool[q].second;
      B->pool.erase(B->pool.begin() + (long)q);
      return 0;
    }
  while (B->resident + bytes > B->budget && !B->pool.empty()) {
    (void)hipFree(B->pool.back().second);
    B->resident -= B->pool.back().first;
    B->pool.pop_back();
  }
  void* p = nullptr;
  HIP_TRY(hipMalloc(&p, bytes));
  B->resident += bytes;
  *out = p;
  return 0;
}

// memory the budget still allows for a new table: pooled buffers count as free
static uint64_t batch_free_bytes(const cdfci_batch* B) {
  uint64_t pooled = 0;
  for (const auto& pb : B->pool) pooled += pb.first;
  const uint64_t used = B->resident - pooled;
  return used >= B->budget ? 0 : B->budget - used;
}

int cdfci_free_batch(cdfci_batch* B) {
  if (!B) return 0;
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  for (int i = 0; i < B->count; ++i) batch_release(B, i);
  void* bufs[] = {B->d_inst, B->d_active, B->d_queue, B->d_elems, B->d_res};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  if (B->ev0) (void)hipEventDestroy(B->ev0);
  if (B->ev1) (void)hipEventDestroy(B->ev1);
  for (auto& pb : B->pool) (void)hipFree(pb.second);
  for (void* t : B->table_of)
    if (t) (void)hipFree(t);
  if (B->own_stream && B->stream) (void)hipStreamDestroy(B->stream);
  delete B;
  return 0;
}

// table slots of every instance from the options (FCI dimension / load factor,
// capped by max_table_slots and by the budget)
static void batch_plan(cdfci_batch* B) {
  const cdfci_batch_opts& o = B->opts;
  for (int i = 0; i < B->count; ++i) {
    const cdfci_hubbard_spec& sp = B->specs[i];
    uint64_t slots = o.table_slots;
    if (!slots) {
      int L = 1;
      for (int k = 0; k < sp.ndim; ++k) L *= sp.dims[k];
      // FCI dimension C(L, na) C(L, nb) as a double (only its size matters)
      double dim = 1.0;
      for (int k = 0; k < sp.n_alpha; ++k) dim = dim * (L - k) / (k + 1);
      for (int k = 0; k < sp.n_beta; ++k) dim = dim * (L - k) / (k + 1);
      slots = 1024;
      while ((double)slots * o.load_factor < dim && slots < (1ull << 40)) slots <<= 1;
      if (o.max_table_slots && slots > o.max_table_slots) slots = o.max_table_slots;
    }
    while (slots > 1024 && slots * sizeof(Slot) > B->budget) slots >>= 1;
    B->slots[i] = slots;
  }
}

// results of the resident instances into B->res (steps counted since init)
static int batch_gather(cdfci_batch* B) {
  std::vector<unsigned> ids;
  for (int i = 0; i < B->count; ++i)
    if (B->ctx[i]) ids.push_back((unsigned)i);
  if (ids.empty()) return 0;
  const int n = (int)ids.size();
  std::vector<HubResult> r((size_t)n);
  HIP_TRY(hipMemcpyAsync(B->d_active, ids.data(), n * sizeof(unsigned), hipMemcpyHostToDevice, B->stream));
  k_hub_results<<<(n + 255) / 256, 256, 0, B->stream>>>(B->d_inst, B->d_active, n, B->d_res);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(r.data(), B->d_res, n * sizeof(HubResult), hipMemcpyDeviceToHost, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  for (int k = 0; k < n; ++k) {
    HubResult x = r[(size_t)k];
    x.steps += B->base_steps[ids[k]];
    B->res[ids[k]] = x;
  }
  return 0;
}

// create (or restore from its checkpoint) instance i and make it resident
static int batch_admit(cdfci_batch* B, int i) {
  const cdfci_batch_opts& o = B->opts;
  const cdfci_hubbard_spec& sp = B->specs[i];
  cdfci_opts co;
  memset(&co, 0, sizeof(co));
  co.table_slots = B->slots[i];
  co.load_factor = o.load_factor;
  co.z_threshold = o.z_threshold;
  co.dx_damping = o.dx_damping;
  co.dx_threshold = o.dx_threshold;
  co.stream = B->stream;
  void* table = nullptr;
  int rc = batch_table(B, batch_bytes(B, i), &table);
  if (rc) return rc;
  co.workspace = table;
  co.workspace_bytes = batch_bytes(B, i);
  cdfci_ctx* c = nullptr;
  rc = cdfci_init_hubbard(sp.dims, sp.ndim, sp.t, sp.U, sp.n_alpha, sp.n_beta, &co, &c);
  if (rc == 0 && !B->ck_keys[i].empty()) {
    rc = cdfci_load(c, B->ck_keys[i].data(), B->ck_c[i].data(), (int64_t)B->ck_c[i].size());
    if (rc == 0) ++B->restarts;
  }
  if (rc) {
    if (c) cdfci_free(c);
    B->pool.push_back({batch_bytes(B, i), table});
    if (rc == CDFCI_ERR_HIP || rc == CDFCI_ERR_INVALID_ARG) return rc;
    B->res[i].error = rc == CDFCI_ERR_TABLE_FULL ? kErrTableFull : kErrNumeric;
    B->init_error[i] = rc;
    return 0;
  }
  B->ck_keys[i].clear();
  B->ck_keys[i].shrink_to_fit();
  B->ck_c[i].clear();
  B->ck_c[i].shrink_to_fit();
  B->ctx[i] = c;
  B->table_of[i] = table;
  B->peak = std::max(B->peak, B->resident);
  HubInst& hi = B->h_inst[i];
  hi.T = c->T;
  hi.mask = c->mask;
  hi.max_entries = c->max_entries;
  hi.ctl = c->ctl;
  hi.step_limit = 0;
  HIP_TRY(hipMemcpyAsync(B->d_inst + i, &hi, sizeof(HubInst), hipMemcpyHostToDevice, B->stream));
  return 0;
}

// make room by releasing a resident instance that is not in `keep`: a
// finished one outright, a running one after checkpointing its (key, c) list
static int batch_evict_one(cdfci_batch* B, const std::vector<char>& keep, bool* done) {
  *done = false;
  int victim = -1;
  for (int pass = 0; pass < 2 && victim < 0; ++pass)
    for (int i = 0; i < B->count; ++i) {
      if (!B->ctx[i] || keep[i]) continue;
      const bool finished = B->res[i].error || B->res[i].stopped;
      if (pass == 0 ? finished : true) {
        victim = i;
        break;
      }
    }
  if (victim < 0) return 0;
  const int i = victim;
  if (!(B->res[i].error || B->res[i].stopped)) {
    // the checkpoint is the wavefunction: the entries with c != 0
    const int rc = export_support(B->ctx[i], B->ck_keys[i], B->ck_c[i]);
    if (rc) return rc;
    B->base_steps[i] = B->res[i].steps;  // a restart counts from zero again
  }
  batch_release(B, i);
  *done = true;
  return 0;
}

static HubArgs batch_args(const cdfci_batch* B, int n_active) {
  HubArgs a;
  a.inst = B->d_inst;
  a.active = B->d_active;
  a.n_inst = n_active;
  a.queue = B->d_queue;
  a.chunk = B->opts.chunk_steps;
  a.tau = B->opts.z_threshold;
  a.theta = B->opts.dx_damping;
  a.dx_tol = B->opts.dx_threshold;
  a.trace_inst = -1;
  a.tr_E = nullptr;
  a.tr_a = nullptr;
  a.tr_b = nullptr;
  return a;
}

// run the resident instances `ids` until each has stopped, failed or used
// nsteps iterations; the replayed graph is captured for this wave's size
static int batch_run_wave(cdfci_batch* B, const std::vector<unsigned>& ids, int64_t nsteps, int* replays) {
  hipStream_t s = B->stream;
  const int n = (int)ids.size();
  if (n == 0 || nsteps <= 0) return 0;
  for (unsigned i : ids)
    if (B->ctx[i]->mode == 1) {  // stepped with k > 1 through its context: fold and reselect
      const int e = enter_single(B->ctx[i]);
      if (e) return e;
    }
  HIP_TRY(hipMemcpyAsync(B->d_active, ids.data(), n * sizeof(unsigned), hipMemcpyHostToDevice, s));
  k_hub_limits<<<(n + 255) / 256, 256, 0, s>>>(B->d_inst, B->d_active, n, nsteps);
  HIP_TRY(hipGetLastError());
  const int R = B->opts.launches_per_graph;
  const int waves = std::min(B->waves, n);
  if (!B->exec || B->graph_n != n || B->graph_waves != waves) {
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    const HubArgs a = batch_args(B, n);
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < R; ++r) {
      k_hub_reset<<<1, 1, 0, s>>>(B->d_queue);
      k_hub_batch<<<waves, 64, 0, s>>>(a);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) {
      g_last_error = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
      return CDFCI_ERR_HIP;
    }
    B->graph = g;
    HIP_TRY(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->graph_n = n;
    B->graph_waves = waves;
  }
  // every visit of a running instance advances it by min(chunk, budget left)
  // steps, so the budget is spent within this many replays
  const int64_t visits = (nsteps + B->opts.chunk_steps - 1) / B->opts.chunk_steps;
  const int64_t max_replays = (visits + R - 1) / R + 1;
  for (int64_t it = 0; it < max_replays; ++it) {
    HIP_TRY(hipGraphLaunch(B->exec, s));
    ++*replays;
    unsigned active = 0;
    HIP_TRY(hipMemcpyAsync(&active, B->d_queue + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (active == 0) break;
  }
  return 0;
}

// one scheduled pass: every instance in `want` (with work left) runs once
static int batch_schedule(cdfci_batch* B, const std::vector<char>& want, int64_t nsteps, int* replays,
                          int* rounds) {
  std::vector<char> pending(want);
  for (;;) {
    std::vector<char> wave((size_t)B->count, 0);
    std::vector<unsigned> ids;
    bool any = false;
    for (int i = 0; i < B->count; ++i) {
      if (!pending[i]) continue;
      if (B->res[i].error || B->res[i].stopped) {
        pending[i] = 0;
        continue;
      }
      any = true;
      if (B->ctx[i]) {
        wave[i] = 1;
        ids.push_back((unsigned)i);
      }
    }
    if (!any) break;
    // admit in index order while the tables fit, evicting instances outside
    // this call's remaining work (finished ones first)
    for (int i = 0; i < B->count; ++i) {
      if (!pending[i] || B->ctx[i] || B->res[i].error) continue;
      const uint64_t need = batch_bytes(B, i);
      bool fits = need <= batch_free_bytes(B);
      while (!fits) {
        std::vector<char> keep(pending);
        for (int j = 0; j < B->count; ++j) keep[j] |= wave[j];
        bool done = false;
        const int rc = batch_evict_one(B, keep, &done);
        if (rc) return rc;
        if (!done) break;
        fits = need <= batch_free_bytes(B);
      }
      if (!fits) break;  // the rest waits for the next wave
      const int rc = batch_admit(B, i);
      if (rc) return rc;
      if (B->ctx[i]) {
        wave[i] = 1;
        ids.push_back((unsigned)i);
      } else {
        pending[i] = 0;  // its start failed: marked in its results
      }
    }
    if (ids.empty()) {
      // nothing resident has work and nothing fits: only pending instances
      // hold memory, so a table larger than the budget is left
      bool stuck = false;
      for (int i = 0; i < B->count; ++i) stuck |= pending[i] && !B->res[i].error && !B->res[i].stopped;
      if (stuck) return CDFCI_ERR_WORKSPACE;
      break;
    }
    std::sort(ids.begin(), ids.end());
    int rc = batch_run_wave(B, ids, nsteps, replays);
    if (rc) return rc;
    ++*rounds;
    rc = batch_gather(B);
    if (rc) return rc;
    for (unsigned i : ids) pending[i] = 0;
  }
  return 0;
}

int cdfci_init_hubbard_batch(const cdfci_hubbard_spec* specs, int count, const cdfci_batch_opts* opts,
                             cdfci_batch** out) {
  if (!out) return CDFCI_ERR_INVALID_ARG;
  *out = nullptr;
  if (!specs || count < 1) return CDFCI_ERR_INVALID_ARG;
  cdfci_batch_opts o;
  memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  if (o.load_factor <= 0.0) o.load_factor = 0.79;
  if (o.dx_damping <= 0.0) o.dx_damping = 0.9;
  if (o.chunk_steps <= 0) o.chunk_steps = 1024;
  if (o.launches_per_graph <= 0) o.launches_per_graph = 4;
  if (o.waves <= 0) o.waves = std::min(count, 8192);
  if ((o.table_slots & (o.table_slots - 1)) != 0 || (o.max_table_slots & (o.max_table_slots - 1)) != 0 ||
      (o.table_slots && o.table_slots < 64) || (o.max_table_slots && o.max_table_slots < 1024) ||
      o.load_factor > 0.95 || o.launches_per_graph > 64)
    return CDFCI_ERR_INVALID_ARG;
  // every spec is checked before any device work
  for (int i = 0; i < count; ++i) {
    const cdfci_hubbard_spec& sp = specs[i];
    if (sp.ndim < 1 || sp.ndim > 3) return CDFCI_ERR_INVALID_ARG;
    int L = 1;
    for (int k = 0; k < sp.ndim; ++k) {
      if (sp.dims[k] < 1 || sp.dims[k] > kMaxOrb) return CDFCI_ERR_INVALID_ARG;
      L *= sp.dims[k];
      if (L > kMaxOrb) return CDFCI_ERR_UNSUPPORTED;
    }
    if (sp.n_alpha < 0 || sp.n_beta < 0 || sp.n_alpha > L || sp.n_beta > L) return CDFCI_ERR_UNSUPPORTED;
    if (sp.n_alpha + sp.n_beta < 1) return CDFCI_ERR_INVALID_ARG;
    if ((int)lattice_bonds(sp.dims, sp.ndim).size() > kHubMaxBonds) return CDFCI_ERR_UNSUPPORTED;
  }
  cdfci_batch* B = new cdfci_batch();
  B->count = count;
  B->opts = o;
  B->waves = o.waves;
  B->specs.assign(specs, specs + count);
  B->ctx.assign(count, nullptr);
  B->table_of.assign(count, nullptr);
  B->slots.assign(count, 0);
  B->res.assign(count, HubResult{0.0, 0, 0, 0, 0, 0});
  B->init_error.assign(count, 0);
  B->base_steps.assign(count, 0);
  B->ck_keys.resize(count);
  B->ck_c.resize(count);
  auto fail = [&](int rc) {
    cdfci_free_batch(B);
    return rc;
  };
  if (o.memory_budget) {
    B->budget = o.memory_budget;
  } else {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(CDFCI_ERR_HIP);
    B->budget = (uint64_t)(0.85 * (double)fr);
  }
  if (o.stream) {
    B->stream = (hipStream_t)o.stream;
  } else {
    if (hipStreamCreate(&B->stream) != hipSuccess) return fail(CDFCI_ERR_HIP);
    B->own_stream = true;
  }
  batch_plan(B);
  B->h_inst.resize(count);
  for (int i = 0; i < count; ++i) {
    const cdfci_hubbard_spec& sp = specs[i];
    const std::vector<std::pair<int, int>> bonds = lattice_bonds(sp.dims, sp.ndim);
    HubInst& hi = B->h_inst[i];
    memset(&hi, 0, sizeof(hi));
    hi.t = sp.t;
    hi.U = sp.U;
    hi.nbonds = (int)bonds.size();
    for (size_t k = 0; k < bonds.size(); ++k) {
      hi.bi[k] = (uint8_t)bonds[k].first;
      hi.bj[k] = (uint8_t)bonds[k].second;
    }
  }
  if (hipMalloc(&B->d_elems, count * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&B->d_inst, count * sizeof(HubInst)) != hipSuccess ||
      hipMalloc(&B->d_active, count * sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&B->d_queue, 2 * sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&B->d_res, count * sizeof(HubResult)) != hipSuccess || hipEventCreate(&B->ev0) != hipSuccess ||
      hipEventCreate(&B->ev1) != hipSuccess)
    return fail(CDFCI_ERR_HIP);
  for (int i = 0; i < count; ++i) B->h_inst[i].elements = B->d_elems + i;
  if (hipMemsetAsync(B->d_elems, 0, count * sizeof(unsigned long long), B->stream) != hipSuccess ||
      hipMemcpyAsync(B->d_inst, B->h_inst.data(), count * sizeof(HubInst), hipMemcpyHostToDevice, B->stream) !=
          hipSuccess ||
      hipStreamSynchronize(B->stream) != hipSuccess)
    return fail(CDFCI_ERR_HIP);
  // admit what fits now (the instances' starts), so small batches are resident at once
  std::vector<char> none((size_t)count, 0);
  for (int i = 0; i < count; ++i) {
    if (batch_bytes(B, i) > batch_free_bytes(B)) break;
    const int rc = batch_admit(B, i);
    if (rc) return fail(rc);
  }
  const int rc = batch_gather(B);
  if (rc) return fail(rc);
  *out = B;
  return 0;
}

int cdfci_step_batch(cdfci_batch* B, int64_t max_steps, cdfci_batch_stats* out) {
  if (!B || max_steps < 0) return CDFCI_ERR_INVALID_ARG;
  hipStream_t s = B->stream;
  int rc = batch_gather(B);
  if (rc) return rc;
  const std::vector<HubResult> r0 = B->res;
  const int restarts0 = B->restarts;
  B->peak = B->resident;
  int replays = 0, rounds = 0;
  HIP_TRY(hipEventRecord(B->ev0, s));
  std::vector<char> want((size_t)B->count, 1);
  if (max_steps > 0) rc = batch_schedule(B, want, max_steps, &replays, &rounds);
  if (rc) return rc;
  HIP_TRY(hipEventRecord(B->ev1, s));
  HIP_TRY(hipEventSynchronize(B->ev1));
  rc = batch_gather(B);
  if (rc) return rc;
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, B->ev0, B->ev1));
  if (out) {
    memset(out, 0, sizeof(*out));
    for (int i = 0; i < B->count; ++i) {
      const HubResult& a = r0[(size_t)i];
      const HubResult& b = B->res[(size_t)i];
      out->steps += b.steps - a.steps;
      out->elements += (int64_t)(b.elements - a.elements);
      if (b.error) ++out->failed;
      else if (b.stopped) ++out->stopped;
      else ++out->running;
    }
    out->graph_replays = replays;
    out->rounds = rounds;
    out->restarts = B->restarts - restarts0;
    out->seconds = ms * 1e-3;
    out->peak_bytes = (double)B->peak;
  }
  return 0;
}

int cdfci_batch_results(cdfci_batch* B, double* energy, int64_t* steps, int* status) {
  if (!B) return CDFCI_ERR_INVALID_ARG;
  int rc = batch_gather(B);
  if (rc) return rc;
  for (int i = 0; i < B->count; ++i) {
    const HubResult& r = B->res[(size_t)i];
    if (energy) energy[i] = r.energy;
    if (steps) steps[i] = r.steps;
    if (status) {
      int st = r.stopped ? 1 : 0;
      if (B->init_error[i]) st = B->init_error[i];
      else if (r.error & kErrTableFull) st = CDFCI_ERR_TABLE_FULL;
      else if (r.error) st = CDFCI_ERR_NUMERIC;
      status[i] = st;
    }
  }
  return 0;
}

int cdfci_batch_trace(cdfci_batch* B, int inst, int64_t nsteps, double* energy, uint64_t* sel_alpha,
                      uint64_t* sel_beta) {
  if (!B || inst < 0 || inst >= B->count || nsteps < 0) return CDFCI_ERR_INVALID_ARG;
  hipStream_t s = B->stream;
  int rc = batch_gather(B);
  if (rc) return rc;
  if (!B->ctx[inst]) {
    // a released finished instance has no state left to continue from
    if (B->res[inst].error || B->res[inst].stopped) return CDFCI_ERR_INVALID_ARG;
    std::vector<char> keep((size_t)B->count, 0);
    keep[inst] = 1;
    while (batch_bytes(B, inst) > batch_free_bytes(B)) {
      bool done = false;
      rc = batch_evict_one(B, keep, &done);
      if (rc) return rc;
      if (!done) return CDFCI_ERR_WORKSPACE;
    }
    rc = batch_admit(B, inst);
    if (rc) return rc;
    if (!B->ctx[inst]) return CDFCI_ERR_INVALID_ARG;
    rc = batch_gather(B);
    if (rc) return rc;
  }
  cdfci_ctx* c = B->ctx[inst];
  if (c->mode == 1) {
    rc = enter_single(c);
    if (rc) return rc;
  }
  Ctl h0;
  rc = ctl_read(c, &h0);
  if (rc) return rc;
  const int64_t step0 = h0.steps;  // trace arrays are indexed by the context's step count
  CallBufs bufs;
  double* dE;
  uint64_t *da, *db;
  HIP_TRY(bufs.alloc(&dE, step0 + nsteps));
  HIP_TRY(bufs.alloc(&da, step0 + nsteps));
  HIP_TRY(bufs.alloc(&db, step0 + nsteps));
  const unsigned id = (unsigned)inst;
  HIP_TRY(hipMemcpyAsync(B->d_active, &id, sizeof(unsigned), hipMemcpyHostToDevice, s));
  k_hub_limits<<<1, 256, 0, s>>>(B->d_inst, B->d_active, 1, nsteps);
  HubArgs a = batch_args(B, 1);
  a.trace_inst = inst;
  a.tr_E = dE;
  a.tr_a = da;
  a.tr_b = db;
  const int64_t visits = (nsteps + B->opts.chunk_steps - 1) / B->opts.chunk_steps;
  for (int64_t it = 0; it < visits + 1 && nsteps > 0; ++it) {
    k_hub_reset<<<1, 1, 0, s>>>(B->d_queue);
    k_hub_batch<<<1, 64, 0, s>>>(a);
    HIP_TRY(hipGetLastError());
    unsigned active = 0;
    HIP_TRY(hipMemcpyAsync(&active, B->d_queue + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (active == 0) break;
  }
  Ctl h1;
  rc = ctl_read(c, &h1);
  if (rc) return rc;
  rc = batch_gather(B);
  if (rc) return rc;
  const int64_t done = h1.steps - step0;
  if (done > 0) {
    if (energy) HIP_TRY(hipMemcpy(energy, dE + step0, done * sizeof(double), hipMemcpyDeviceToHost));
    if (sel_alpha) HIP_TRY(hipMemcpy(sel_alpha, da + step0, done * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (sel_beta) HIP_TRY(hipMemcpy(sel_beta, db + step0, done * sizeof(uint64_t), hipMemcpyDeviceToHost));
  }
  return 0;
}

int cdfci_batch_context(cdfci_batch* B, int inst, cdfci_ctx** ctx) {
  if (!B || !ctx || inst < 0 || inst >= B->count) return CDFCI_ERR_INVALID_ARG;
  if (!B->ctx[inst]) return CDFCI_ERR_INVALID_ARG;
  *ctx = B->ctx[inst];
  return 0;
}

int cdfci_batch_tables(cdfci_batch* B, uint64_t* slots) {
  if (!B || !slots) return CDFCI_ERR_INVALID_ARG;
  for (int i = 0; i < B->count; ++i) slots[i] = B->slots[i];
  return 0;
}

int cdfci_tune_k(cdfci_ctx* c, const int* ks, int nk, double seconds_per_trial, int rounds, int* best_k,
                 double* rates) {
  if (!c || !ks || nk < 1 || !best_k || rounds < 1 || !(seconds_per_trial > 0.0)) return CDFCI_ERR_INVALID_ARG;
  for (int i = 0; i < nk; ++i)
    if (ks[i] < 1 || ks[i] > kMaxK) return CDFCI_ERR_INVALID_ARG;
  std::vector<double> sum(nk, 0.0), secs(nk, 0.0);
  // an uncounted first trial: right after a start the energy falls far faster
  // than later, which would favour whichever candidate ran first
  for (int r = -1; r < rounds; ++r) {
    for (int q = 0; q < nk; ++q) {
      const int i = (r & 1) ? nk - 1 - q : q;
      const int k = ks[i];
      double E0 = 0.0, E1 = 0.0, t = 0.0;
      int rc = cdfci_energy(c, 0, &E0);
      if (rc) return rc;
      int64_t n = 1;
      for (int guard = 0; guard < 64 && t < seconds_per_trial; ++guard) {
        cdfci_stats st;
        rc = cdfci_step(c, k, n, &st);
        if (rc) return rc;
        t += st.seconds;
        if (st.stopped || st.steps < n) break;
        const double per = st.seconds / (double)std::max<int64_t>(1, st.steps);
        const double left = seconds_per_trial - t;
        n = std::max<int64_t>(1, std::min<int64_t>((int64_t)(left / std::max(per, 1e-7)), 4 * n));
      }
      rc = cdfci_energy(c, 0, &E1);
      if (rc) return rc;
      if (r < 0) break;
      sum[i] += E0 - E1;
      secs[i] += t;
    }
  }
  int best = 0;
  for (int i = 0; i < nk; ++i) {
    const double rate = secs[i] > 0.0 ? sum[i] / secs[i] : 0.0;
    if (rates) rates[i] = rate;
    const double rb = secs[best] > 0.0 ? sum[best] / secs[best] : 0.0;
    if (rate > rb) best = i;
  }
  *best_k = ks[best];
  return 0;
}

// a new load factor: every table is re-planned; resident instances are
// checkpointed (running) or released (finished) and restarted at their new size
static int batch_replan(cdfci_batch* B, double lf) {
  std::vector<char> keep((size_t)B->count, 0);
  for (;;) {
    bool done = false;
    const int rc = batch_evict_one(B, keep, &done);
    if (rc) return rc;
    if (!done) break;
  }
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  B->graph_n = -1;
  B->opts.load_factor = lf;
  batch_plan(B);
  return 0;
}

int cdfci_tune_batch(cdfci_batch* B, const int64_t* chunks, int nc, const int* launches, int nl,
                     const double* lfs, int nlf, int64_t steps_per_trial, int64_t* best_chunk, int* best_launches,
                     double* best_lf) {
  if (!B || !chunks || nc < 1 || !launches || nl < 1 || steps_per_trial < 1 || nlf < 0 || (nlf && !lfs))
    return CDFCI_ERR_INVALID_ARG;
  for (int i = 0; i < nc; ++i)
    if (chunks[i] < 1) return CDFCI_ERR_INVALID_ARG;
  for (int i = 0; i < nl; ++i)
    if (launches[i] < 1 || launches[i] > 64) return CDFCI_ERR_INVALID_ARG;
  for (int i = 0; i < nlf; ++i)
    if (!(lfs[i] > 0.0 && lfs[i] <= 0.95)) return CDFCI_ERR_INVALID_ARG;
  std::vector<double> cand_lf;
  if (nlf) cand_lf.assign(lfs, lfs + nlf);
  else cand_lf.push_back(B->opts.load_factor);
  double best_rate = -1.0;
  int64_t bc = B->opts.chunk_steps;
  int bl = B->opts.launches_per_graph;
  double blf = B->opts.load_factor;
  for (double lf : cand_lf) {
    if (lf != B->opts.load_factor) {
      const int rc = batch_replan(B, lf);
      if (rc) return rc;
    }
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nl; ++j) {
        // a new setting needs a new graph
        if (B->exec) (void)hipGraphExecDestroy(B->exec);
        if (B->graph) (void)hipGraphDestroy(B->graph);
        B->exec = nullptr;
        B->graph = nullptr;
        B->graph_n = -1;
        B->opts.chunk_steps = chunks[i];
        B->opts.launches_per_graph = launches[j];
        cdfci_batch_stats st;
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = cdfci_step_batch(B, steps_per_trial, &st);
        if (rc) return rc;
        const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        const double rate = wall > 0.0 ? (double)st.steps / wall : 0.0;
        if (rate > best_rate) {
          best_rate = rate;
          bc = chunks[i];
          bl = launches[j];
          blf = lf;
        }
      }
  }
  if (blf != B->opts.load_factor) {
    const int rc = batch_replan(B, blf);
    if (rc) return rc;
  }
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  B->graph_n = -1;
  B->opts.chunk_steps = bc;
  B->opts.launches_per_graph = bl;
  if (best_chunk) *best_chunk = bc;
  if (best_launches) *best_launches = bl;
  if (best_lf) *best_lf = blf;
  return 0;
}

const char* cdfci_strerror(int code) {
  switch (code) {
    case CDFCI_OK: return "ok";
    case CDFCI_ERR_INVALID_ARG: return "invalid argument or context state";
    case CDFCI_ERR_UNSUPPORTED: return "unsupported size or mode";
    case CDFCI_ERR_TABLE_FULL: return "hash table full (occupancy limit or probe bound exceeded)";
    case CDFCI_ERR_NOT_NEGATIVE: return "starting energy is not negative";
    case CDFCI_ERR_HIP: return "HIP runtime error";
    case CDFCI_ERR_BARRIER: return "device-wide barrier timed out";
    case CDFCI_ERR_WORKSPACE: return "workspace too small or misaligned";
    case CDFCI_ERR_NUMERIC: return "non-finite value in a multicoordinate step";
    case CDFCI_ERR_INTERNAL: return "internal consistency check failed";
    default: return "unknown error";
  }
}

const char* cdfci_last_error(void) { return g_last_error.c_str(); }

int cdfci_set_timing(cdfci_ctx* c, int on) {
  if (!c) return CDFCI_ERR_INVALID_ARG;
  c->timing = on ? 1 : 0;
  for (double& t : c->t_phase_mc) t = 0.0;
  c->n_timed = 0;
  return 0;
}

int cdfci_mc_phase_times(cdfci_ctx* c, double* seconds, int64_t* steps) {
  if (!c || !seconds) return CDFCI_ERR_INVALID_ARG;
  for (int q = 0; q < 7; ++q) seconds[q] = c->t_phase_mc[q];
  if (steps) *steps = c->n_timed;
  return 0;
}

int cdfci_mc_select_stats(cdfci_ctx* c, int64_t* counts) {
  if (!c || !counts || !c->mst) return CDFCI_ERR_INVALID_ARG;
  McState st;
  HIP_TRY(hipMemcpyAsync(&st, c->mst, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  counts[0] = (int64_t)st.acc_sel;
  counts[1] = (int64_t)st.acc_pos;
  counts[2] = (int64_t)st.acc_kept;
  counts[3] = (int64_t)st.acc_fallback;
  return 0;
}

int cdfci_phase_times(cdfci_ctx* c, double* seconds) {
  if (!c || !seconds) return CDFCI_ERR_INVALID_ARG;
#ifndef CDFCI_PHASE_TIMING
  return CDFCI_ERR_UNSUPPORTED;  // timers compiled out of the kernel
#endif
  Ctl h;
  int rc = ctl_read(c, &h);
  if (rc) return rc;
  int khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
  for (int k = 0; k < 4; ++k) seconds[k] = (double)h.t_phase[k] / (1e3 * (double)khz);
  return 0;
}

}  // extern "C"

// ===========================================================================
// Several low-lying states (xCDFCI, Sec. 3.3): host side.

struct cdfci_xctx {
  cdfci_ctx* base = nullptr;  // integrals, sizes and stream (no single-state table)
  int n = 0;
  double shift = 0.0;
  XKey* K = nullptr;
  double* R = nullptr;
  uint64_t nslots = 0, mask = 0, max_entries = 0;
  XCtl* x = nullptr;
  XPartial* parts = nullptr;
  double* dE = nullptr;
  int grid = 0, block = 256, max_parts = 0;
  int64_t n_col = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool poisoned = false;
  bool grid_fixed = false;
  int kind = 0;  // 0: integrals, 1: momentum-space Hubbard
  HamK hk{};
  double* d_eps = nullptr;
};

namespace {

constexpr int kXSelParts = 4096;

int xctl_read(cdfci_xctx* X, XCtl* h) {
  hipStream_t s = X->base->stream;
  HIP_TRY(hipMemcpyAsync(h, X->x, sizeof(XCtl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int xcheck(cdfci_xctx* X, const XCtl& h) {
  int rc = 0;
  if ((h.error & kErrTableFull) || h.occupied > X->max_entries) rc = CDFCI_ERR_TABLE_FULL;
  else if (h.error & kErrBarrier) rc = CDFCI_ERR_BARRIER;
  else if (h.error) rc = CDFCI_ERR_HIP;
  if (rc) X->poisoned = true;
  return rc;
}

__global__ void k_xbegin(XCtl* x) {
  x->steps_this_call = 0;
  x->arrive = 0;
}

__global__ void k_xfinish(XCtl* x) {
  x->steps += x->steps_this_call;
  x->arrive = 0;
}

const void* x_kernel(int n, int kind) {
#define XITER_CASE(NS) \
  case NS:             \
    return kind ? (const void*)k_xiter<NS, 1> : (const void*)k_xiter<NS, 0>;
  switch (n) {
    XITER_CASE(1)
    XITER_CASE(2)
    XITER_CASE(3)
    XITER_CASE(4)
    XITER_CASE(5)
    XITER_CASE(6)
    XITER_CASE(7)
    default:
      return kind ? (const void*)k_xiter<8, 1> : (const void*)k_xiter<8, 0>;
  }
#undef XITER_CASE
}

// one cooperative launch of A.nsteps iterations; the grid (one lane per
// column entry, fewer workgroups if not all fit at once) must be resident
int x_launch(cdfci_xctx* X, XArgs& A) {
  hipStream_t s = X->base->stream;
  const void* fn = x_kernel(X->n, X->kind);
  if (!X->grid_fixed) {
    int cus = 0, per_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, X->base->device));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, X->block, 0));
    X->grid = std::max(1, std::min(X->grid, std::min(std::max(1, per_cu) * cus, X->max_parts / 2)));
    X->grid_fixed = true;
  }
  void* args[] = {&A};
  HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(X->grid), dim3(X->block), args, 0, s));
  return 0;
}

// table, control block and buffers for n_col-entry columns
int x_alloc(cdfci_xctx* X) {
  cdfci_ctx* c = X->base;
  const cdfci_opts& o = c->opts;
  const int n = X->n;
  hipStream_t s = c->stream;
  X->nslots = o.table_slots;
  X->mask = X->nslots - 1;
  X->max_entries = (uint64_t)(o.load_factor * (double)X->nslots);
  X->n_col = X->kind ? column_count_k(c->N, c->na, c->nb) : column_count(c->N, c->na, c->nb);
  // workgroup size: 128 threads while the column (diagonal excluded) still
  // gives every lane one entry with one workgroup per compute unit (a shorter
  // tail of slow probes per workgroup), else 256
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  X->block = (X->n_col - 1 + 127) / 128 <= cus ? 128 : 256;
  X->grid = (int)std::max<int64_t>(1, (X->n_col - 1 + X->block - 1) / X->block);
  X->max_parts = std::max(X->grid, kXSelParts);
  HIP_TRY(hipMalloc(&X->K, X->nslots * sizeof(XKey)));
  HIP_TRY(hipMalloc(&X->R, X->nslots * 2 * n * sizeof(double)));
  HIP_TRY(hipMalloc(&X->x, sizeof(XCtl)));
  HIP_TRY(hipMalloc(&X->parts, X->max_parts * sizeof(XPartial)));
  HIP_TRY(hipMalloc(&X->dE, kXMax * sizeof(double)));
  HIP_TRY(hipEventCreate(&X->ev0));
  HIP_TRY(hipEventCreate(&X->ev1));
  XCtl h0;
  memset(&h0, 0, sizeof(h0));
  h0.n = n;
  h0.shift = X->shift;
  h0.islot = -1;
  HIP_TRY(hipMemcpyAsync(X->x, &h0, sizeof(XCtl), hipMemcpyHostToDevice, s));
  k_xclear<<<2048, 256, 0, s>>>(X->K, X->R, X->nslots, n);
  HIP_TRY(hipGetLastError());
  return 0;
}

// the first coordinate: the stored row of largest |G_j|_inf
int x_first(cdfci_xctx* X) {
  hipStream_t s = X->base->stream;
  const int sel_blocks = (int)std::min<uint64_t>((X->nslots + 255) / 256, (uint64_t)kXSelParts);
  k_xselect_table<<<sel_blocks, 256, 0, s>>>(X->K, X->R, X->nslots, X->x, X->parts);
  k_xselect_final<<<1, 1, 0, s>>>(X->parts, sel_blocks, X->x);
  HIP_TRY(hipGetLastError());
  XCtl h;
  int rc = xctl_read(X, &h);
  if (rc) return rc;
  rc = xcheck(X, h);
  if (rc) return rc;
  if (h.islot < 0) return CDFCI_ERR_INVALID_ARG;
  return 0;
}

// C^(0) at the reference (a0, b0) and its lowest-diagonal connected
// determinants, B^(0), S, Q and the first coordinate
int x_setup(cdfci_xctx* X, uint64_t a0, uint64_t b0) {
  int rc = x_alloc(X);
  if (rc) return rc;
  cdfci_ctx* c = X->base;
  const int n = X->n;
  hipStream_t s = c->stream;
  const Ham H = ham_of(c);
  const int64_t n_col = X->n_col;
  CallBufs bufs;
  double *diag, *coef;
  uint64_t *ka, *kb;
  XInitTask* tasks;
  int* d_found;
  HIP_TRY(bufs.alloc(&diag, n_col));
  HIP_TRY(bufs.alloc(&ka, n_col));
  HIP_TRY(bufs.alloc(&kb, n_col));
  HIP_TRY(bufs.alloc(&tasks, kXMax));
  HIP_TRY(bufs.alloc(&d_found, 1));
  HIP_TRY(bufs.alloc(&coef, kXMax * kXMax));
  const XInitTask d0{a0, b0};
  double eye[kXMax * kXMax] = {};
  for (int k = 0; k < n; ++k) eye[k * n + k] = 1.0;
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(tasks, &d0, sizeof(d0), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(coef, eye, sizeof(eye), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_found, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  const int cblocks = (int)((n_col + 255) / 256);
  k_xconn_diag<<<cblocks, 256, 0, s>>>(H, a0, b0, n_col, diag, ka, kb);
  k_xconn_rank<<<cblocks, 256, 0, s>>>(diag, ka, kb, n_col, n, tasks, d_found);
  HIP_TRY(hipGetLastError());
  int found = 0;
  HIP_TRY(hipMemcpyAsync(&found, d_found, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (found != n - 1) return CDFCI_ERR_UNSUPPORTED;
  const int m = n;
  k_xinit_insert<<<(m + 63) / 64, 64, 0, s>>>(X->K, X->R, X->mask, tasks, coef, m, n, X->x);
  const int chunks = (int)std::min<int64_t>(cblocks, 1024);
  k_xinit_scatter<<<dim3(chunks, m), 256, 0, s>>>(H, X->K, X->R, X->mask, tasks, coef, n, n_col, X->shift,
                                                   X->x);
  k_xinit_matrices<<<1, 1, 0, s>>>(X->K, X->R, X->mask, tasks, m, n, X->x);
  HIP_TRY(hipGetLastError());
  return x_first(X);
}

int x_create(int N, int na, int nb, int n_states, double shift, const cdfci_opts* opts, cdfci_xctx** out,
             cdfci_xctx** X) {
  if (!out) return CDFCI_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_states < 1 || n_states > kXMax || !std::isfinite(shift)) return CDFCI_ERR_INVALID_ARG;
  cdfci_ctx* base = nullptr;
  int rc = make_ctx(N, na, nb, opts, &base);
  if (rc) return rc;
  *X = new cdfci_xctx();
  (*X)->base = base;
  (*X)->n = n_states;
  (*X)->shift = shift;
  return 0;
}

}  // namespace

extern "C" {

int cdfci_xfree(cdfci_xctx* X) {
  if (!X) return 0;
  if (X->base) {
    if (X->base->stream) (void)hipStreamSynchronize(X->base->stream);
    else (void)hipDeviceSynchronize();
  }
  void* bufs[] = {X->K, X->R, X->x, X->parts, X->dE, X->d_eps};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  if (X->ev0) (void)hipEventDestroy(X->ev0);
  if (X->ev1) (void)hipEventDestroy(X->ev1);
  cdfci_free(X->base);
  delete X;
  return 0;
}

int cdfci_xinit(const double* h, const double* eri, int n_orb, int n_alpha, int n_beta, int n_states,
                double shift, const cdfci_opts* opts, cdfci_xctx** out) {
  if (!h || !eri) return CDFCI_ERR_INVALID_ARG;
  cdfci_xctx* X = nullptr;
  int rc = x_create(n_orb, n_alpha, n_beta, n_states, shift, opts, out, &X);
  if (rc) return rc;
  rc = upload(X->base, h, eri);
  uint64_t a0 = 0, b0 = 0;
  if (X->base->opts.init_kind == 2) {  // alternating chain pattern
    for (int p = 0, k = 0; p < n_orb && k < n_alpha; p += 2, ++k) a0 |= 1ull << p;
    for (int p = 1, k = 0; p < n_orb && k < n_beta; p += 2, ++k) b0 |= 1ull << p;
  } else {  // aufbau: the lowest h_pp (ties: the lower index)
    std::vector<int> order(n_orb);
    for (int p = 0; p < n_orb; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(),
                     [&](int p, int q) { return h[(size_t)p * n_orb + p] < h[(size_t)q * n_orb + q]; });
    for (int k = 0; k < n_alpha; ++k) a0 |= 1ull << order[k];
    for (int k = 0; k < n_beta; ++k) b0 |= 1ull << order[k];
  }
  if (!rc) rc = x_setup(X, a0, b0);
  if (rc) {
    cdfci_xfree(X);
    return rc;
  }
  *out = X;
  return 0;
}

int cdfci_xinit_hubbard(const int* dims, int ndim, double t, double U, int n_alpha, int n_beta,
                        int n_states, double shift, const cdfci_opts* opts, cdfci_xctx** out) {
  if (!dims || ndim < 1 || ndim > 3 || !out) return CDFCI_ERR_INVALID_ARG;
  int L = 1;
  for (int i = 0; i < ndim; ++i) {
    if (dims[i] < 1) return CDFCI_ERR_INVALID_ARG;
    L *= dims[i];
  }
  if (L > kMaxOrb) return CDFCI_ERR_UNSUPPORTED;
  cdfci_xctx* X = nullptr;
  int rc = x_create(L, n_alpha, n_beta, n_states, shift, opts, out, &X);
  if (rc) return rc;
  std::vector<double> h, eri;
  hubbard_integrals(dims, ndim, t, U, h, eri);
  rc = upload(X->base, h.data(), eri.data());
  uint64_t a0 = 0, b0 = 0;
  neel_determinant(dims, ndim, n_alpha, n_beta, &a0, &b0);
  if (!rc) rc = x_setup(X, a0, b0);
  if (rc) {
    cdfci_xfree(X);
    return rc;
  }
  *out = X;
  return 0;
}

int cdfci_xenergies(cdfci_xctx* X, double* energies) {
  if (!X || !energies) return CDFCI_ERR_INVALID_ARG;
  hipStream_t s = X->base->stream;
  k_xenergies<<<1, 1, 0, s>>>(X->x, X->dE);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(energies, X->dE, X->n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int cdfci_xstep(cdfci_xctx* X, int64_t nsteps, double* energies, uint64_t* sel_alpha, uint64_t* sel_beta,
                cdfci_stats* out) {
  if (!X || X->poisoned || nsteps < 0) return CDFCI_ERR_INVALID_ARG;
  XCtl before;
  int rc = xctl_read(X, &before);
  if (rc) return rc;
  if (before.islot < 0 || (uint64_t)before.islot >= X->nslots) return CDFCI_ERR_INVALID_ARG;
  const int n = X->n;
  CallBufs bufs;
  XArgs A;
  memset(&A, 0, sizeof(A));
  double* dE = nullptr;
  if (energies) {
    HIP_TRY(bufs.alloc(&A.tr_SQ, (uint64_t)nsteps * 2 * n * n));
    HIP_TRY(bufs.alloc(&dE, (uint64_t)nsteps * n));
  }
  if (sel_alpha) HIP_TRY(bufs.alloc(&A.tr_a, (uint64_t)nsteps));
  if (sel_beta) HIP_TRY(bufs.alloc(&A.tr_b, (uint64_t)nsteps));
  A.H = ham_of(X->base);
  A.HK = X->hk;
  A.K = X->K;
  A.R = X->R;
  A.mask = X->mask;
  A.max_entries = X->max_entries;
  A.x = X->x;
  A.parts = X->parts;
  A.n_col = X->n_col;
  A.tau = X->base->opts.z_threshold;
  A.theta = X->base->opts.dx_damping;
  A.dx_tol = X->base->opts.dx_threshold;
  hipStream_t s = X->base->stream;
  A.nsteps = nsteps;
  k_xbegin<<<1, 1, 0, s>>>(X->x);
  HIP_TRY(hipEventRecord(X->ev0, s));
  if (nsteps > 0) {
    rc = x_launch(X, A);
    if (rc) return rc;
  }
  HIP_TRY(hipEventRecord(X->ev1, s));
  k_xfinish<<<1, 1, 0, s>>>(X->x);
  HIP_TRY(hipGetLastError());
  XCtl h;
  rc = xctl_read(X, &h);
  if (rc) return rc;
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, X->ev0, X->ev1));
  const int64_t done = h.steps_this_call;
  if (energies && done) {
    k_xtrace_energies<<<(unsigned)((done + 63) / 64), 64, 0, s>>>(A.tr_SQ, done, n, X->shift, dE);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(energies, dE, (size_t)done * n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (sel_alpha && done) HIP_TRY(hipMemcpy(sel_alpha, A.tr_a, done * sizeof(uint64_t), hipMemcpyDeviceToHost));
  if (sel_beta && done) HIP_TRY(hipMemcpy(sel_beta, A.tr_b, done * sizeof(uint64_t), hipMemcpyDeviceToHost));
  rc = xcheck(X, h);
  if (out) {
    double E[kXMax];
    int e = cdfci_xenergies(X, E);
    if (e) return e;
    out->steps = done;
    out->total_steps = h.steps;
    out->elements = done * X->n_col;
    out->inserts = (int64_t)(h.inserts - before.inserts);
    out->probes = 0;
    out->atomics = 0;
    out->occupied = h.occupied;
    out->max_probe = h.max_probe;
    out->stopped = h.stopped;
    out->energy = E[0];
    out->dx = h.d;
    double ts = 0.0, tq = 0.0;
    for (int k = 0; k < n; ++k) {
      ts += h.S_hi[k * n + k] + h.S_lo[k * n + k];
      tq += h.Q_hi[k * n + k] + h.Q_lo[k * n + k];
    }
    out->mu = ts;
    out->alpha = tq;
    out->seconds = ms * 1e-3;
  }
  return rc;
}

int cdfci_xmatrices(cdfci_xctx* X, double* S, double* Q) {
  if (!X) return CDFCI_ERR_INVALID_ARG;
  XCtl h;
  int rc = xctl_read(X, &h);
  if (rc) return rc;
  for (int k = 0; k < X->n * X->n; ++k) {
    if (S) S[k] = h.S_hi[k] + h.S_lo[k];
    if (Q) Q[k] = h.Q_hi[k] + h.Q_lo[k];
  }
  return 0;
}

int cdfci_xexport(cdfci_xctx* X, uint64_t* keys, double* C, double* B, int64_t cap, int64_t* count) {
  if (!X || !count || cap < 0) return CDFCI_ERR_INVALID_ARG;
  XCtl h;
  int rc = xctl_read(X, &h);
  if (rc) return rc;
  const int n = X->n;
  const int64_t m = (int64_t)std::min<uint64_t>(h.occupied, (uint64_t)cap);
  CallBufs bufs;
  uint64_t *da, *db;
  double *dc, *dbv;
  unsigned long long* dcount;
  HIP_TRY(bufs.alloc(&da, m));
  HIP_TRY(bufs.alloc(&db, m));
  HIP_TRY(bufs.alloc(&dc, (uint64_t)m * n));
  HIP_TRY(bufs.alloc(&dbv, (uint64_t)m * n));
  HIP_TRY(bufs.alloc(&dcount, 1));
  hipStream_t s = X->base->stream;
  HIP_TRY(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), s));
  k_xexport<<<1024, 256, 0, s>>>(X->K, X->R, X->nslots, n, da, db, dc, dbv, m, dcount);
  HIP_TRY(hipGetLastError());
  unsigned long long total = 0;
  HIP_TRY(hipMemcpyAsync(&total, dcount, sizeof(total), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *count = (int64_t)total;
  const int64_t w = std::min<int64_t>((int64_t)total, m);
  if (w > 0) {
    std::vector<uint64_t> ha(w), hb(w);
    HIP_TRY(hipMemcpy(ha.data(), da, w * sizeof(uint64_t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hb.data(), db, w * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (keys)
      for (int64_t i = 0; i < w; ++i) {
        keys[2 * i] = ha[i];
        keys[2 * i + 1] = hb[i];
      }
    if (C) HIP_TRY(hipMemcpy(C, dc, (size_t)w * n * sizeof(double), hipMemcpyDeviceToHost));
    if (B) HIP_TRY(hipMemcpy(B, dbv, (size_t)w * n * sizeof(double), hipMemcpyDeviceToHost));
  }
  return 0;
}

}  // extern "C"

// ===========================================================================
// OptOrbFCI (Sec. 3.4, Alg. 4): host side.  The FCI solves are ordinary
// contexts (cdfci_init, cdfci_step, cdfci_rdm_backward); the four-index
// transforms, P4 and its two-body gradient run on the device; the N x N
// algebra of the projected steps (polar factor) stays on the host.

namespace {

// eigenvalues w and eigenvectors (columns of V) of the symmetric n x n A by
// cyclic Jacobi
void host_sym_eig(std::vector<double> A, int n, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        if (i != j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double theta = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

// polar factor X (X^T X)^(-1/2) of the M x N matrix X (row-major)
bool host_orth(const std::vector<double>& X, int M, int N, std::vector<double>& out) {
  std::vector<double> G((size_t)N * N, 0.0), w, V;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int a = 0; a < M; ++a) s += X[(size_t)a * N + i] * X[(size_t)a * N + j];
      G[(size_t)i * N + j] = s;
    }
  host_sym_eig(G, N, w, V);
  std::vector<double> R((size_t)N * N, 0.0);  // (X^T X)^(-1/2)
  for (int k = 0; k < N; ++k) {
    if (!(w[k] > 0.0)) return false;
    const double f = 1.0 / std::sqrt(w[k]);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) R[(size_t)i * N + j] += V[(size_t)i * N + k] * f * V[(size_t)j * N + k];
  }
  out.assign((size_t)M * N, 0.0);
  for (int a = 0; a < M; ++a)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int i = 0; i < N; ++i) s += X[(size_t)a * N + i] * R[(size_t)i * N + j];
      out[(size_t)a * N + j] = s;
    }
  return true;
}

struct OrbWork {
  int M = 0, N = 0;
  hipStream_t s = nullptr;
  CallBufs bufs;
  double *eri = nullptr, *U = nullptr, *t1 = nullptr, *t2 = nullptr, *W = nullptr, *eri2 = nullptr;
  double *Gs = nullptr, *grad2 = nullptr, *part = nullptr;
  std::vector<double> h, g1;  // M x M; N x N (gamma)
  std::vector<double> G2;     // Gamma (N^4), as the reverse pass returns it
};

constexpr int kOrbDotBlocks = 256;

// W = eri with positions 1..3 rotated (M x N^3), then eri' (N^4) into w.eri2
int orb_transform(OrbWork& w) {
  const int M = w.M, N = w.N;
  auto launch = [&](const double* in, double* out, int d0, int d1, int d2, int d3, int pos) {
    int64_t tot = (int64_t)d0 * d1 * d2 * d3 / (pos == 0 ? d0 : pos == 1 ? d1 : pos == 2 ? d2 : d3) * N;
    k_orb_contract<<<(unsigned)((tot + 255) / 256), 256, 0, w.s>>>(in, out, w.U, M, N, d0, d1, d2, d3, pos);
  };
  launch(w.eri, w.t1, M, M, M, M, 1);  // M N M M
  launch(w.t1, w.t2, M, N, M, M, 2);   // M N N M
  launch(w.t2, w.W, M, N, N, M, 3);    // M N N N
  launch(w.W, w.eri2, M, N, N, N, 0);  // N N N N
  HIP_TRY(hipGetLastError());
  return 0;
}

// P4(U) and its gradient (M x N) for the U already on the device
int orb_eval(OrbWork& w, const std::vector<double>& U, double* value, std::vector<double>& grad) {
  const int M = w.M, N = w.N;
  HIP_TRY(hipMemcpyAsync(w.U, U.data(), (size_t)M * N * sizeof(double), hipMemcpyHostToDevice, w.s));
  int rc = orb_transform(w);
  if (rc) return rc;
  const int64_t n4 = (int64_t)N * N * N * N;
  k_orb_dot<<<kOrbDotBlocks, 256, 0, w.s>>>(w.eri2, w.Gs, n4, w.part);
  k_orb_grad2<<<(unsigned)(M * N), 256, 0, w.s>>>(w.W, w.Gs, M, N, w.grad2);
  HIP_TRY(hipGetLastError());
  std::vector<double> part(kOrbDotBlocks);
  grad.assign((size_t)M * N, 0.0);
  HIP_TRY(hipMemcpyAsync(part.data(), w.part, kOrbDotBlocks * sizeof(double), hipMemcpyDeviceToHost, w.s));
  HIP_TRY(hipMemcpyAsync(grad.data(), w.grad2, (size_t)M * N * sizeof(double), hipMemcpyDeviceToHost, w.s));
  HIP_TRY(hipStreamSynchronize(w.s));
  double two = 0.0;
  for (double p : part) two += p;
  // one-body part: h' = U^T h U against gamma, gradient h U (gamma + gamma^T)
  std::vector<double> hU((size_t)M * N, 0.0);
  for (int a = 0; a < M; ++a)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int b = 0; b < M; ++b) s += w.h[(size_t)a * M + b] * U[(size_t)b * N + j];
      hU[(size_t)a * N + j] = s;
    }
  double one = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double hij = 0.0;
      for (int a = 0; a < M; ++a) hij += U[(size_t)a * N + i] * hU[(size_t)a * N + j];
      one += hij * w.g1[(size_t)i * N + j];
    }
  for (int a = 0; a < M; ++a)
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int j = 0; j < N; ++j) s += hU[(size_t)a * N + j] * (w.g1[(size_t)j * N + i] + w.g1[(size_t)i * N + j]);
      grad[(size_t)a * N + i] += s;
    }
  *value = one + 0.5 * two;
  return 0;
}

double frob_dot(const std::vector<double>& x, const std::vector<double>& y) {
  double s = 0.0;
  for (size_t k = 0; k < x.size(); ++k) s += x[k] * y[k];
  return s;
}

// norm of the Riemannian gradient G - U sym(U^T G)
double riemannian_norm(const std::vector<double>& U, const std::vector<double>& G, int M, int N) {
  std::vector<double> S((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int a = 0; a < M; ++a) s += U[(size_t)a * N + i] * G[(size_t)a * N + j];
      S[(size_t)i * N + j] = s;
    }
  double n2 = 0.0;
  for (int a = 0; a < M; ++a)
    for (int j = 0; j < N; ++j) {
      double r = G[(size_t)a * N + j];
      for (int i = 0; i < N; ++i) r -= U[(size_t)a * N + i] * 0.5 * (S[(size_t)i * N + j] + S[(size_t)j * N + i]);
      n2 += r * r;
    }
  return std::sqrt(n2);
}

}  // namespace

extern "C" int cdfci_optorb(const double* h, const double* eri, int M, int n_alpha, int n_beta,
                            const cdfci_optorb_opts* opts, double* U_io, double* energies, double* p4_values,
                            int* n_outer) {
  if (!h || !eri || !opts || !U_io || !n_outer) return CDFCI_ERR_INVALID_ARG;
  cdfci_optorb_opts o = *opts;
  const int N = o.n_active;
  if (M < 1 || N < 1 || N > M || N > kMaxOrb || n_alpha < 0 || n_beta < 0 || n_alpha > N || n_beta > N ||
      n_alpha + n_beta < 1)
    return CDFCI_ERR_INVALID_ARG;
  if (o.max_outer <= 0) o.max_outer = 20;
  if (o.max_inner <= 0) o.max_inner = 100;
  if (o.k <= 0) o.k = 1;
  if (o.cd_steps <= 0) o.cd_steps = 1000000;
  if (o.cd_dx_threshold <= 0.0) o.cd_dx_threshold = 1e-10;
  if (o.energy_tol == 0.0) o.energy_tol = 1e-8;
  if (o.grad_tol <= 0.0) o.grad_tol = 1e-8;
  if (o.step0 <= 0.0) o.step0 = 1e-2;
  if (o.table_slots == 0) o.table_slots = 1ull << 22;
  OrbWork w;
  w.M = M;
  w.N = N;
  w.s = (hipStream_t)o.stream;
  w.h.assign(h, h + (size_t)M * M);
  const size_t m4 = (size_t)M * M * M * M, n4 = (size_t)N * N * N * N;
  HIP_TRY(w.bufs.alloc(&w.eri, m4));
  HIP_TRY(w.bufs.alloc(&w.U, (uint64_t)M * N));
  HIP_TRY(w.bufs.alloc(&w.t1, (uint64_t)M * N * M * M));
  HIP_TRY(w.bufs.alloc(&w.t2, (uint64_t)M * N * N * M));
  HIP_TRY(w.bufs.alloc(&w.W, (uint64_t)M * N * N * N));
  HIP_TRY(w.bufs.alloc(&w.eri2, n4));
  HIP_TRY(w.bufs.alloc(&w.Gs, n4));
  HIP_TRY(w.bufs.alloc(&w.grad2, (uint64_t)M * N));
  HIP_TRY(w.bufs.alloc(&w.part, kOrbDotBlocks));
  HIP_TRY(hipMemcpyAsync(w.eri, eri, m4 * sizeof(double), hipMemcpyHostToDevice, w.s));
  std::vector<double> U((size_t)M * N, 0.0);
  if (o.have_u) {
    U.assign(U_io, U_io + (size_t)M * N);
    std::vector<double> Uo;
    if (!host_orth(U, M, N, Uo)) return CDFCI_ERR_INVALID_ARG;
    U = Uo;
  } else {  // the identity columns of the N orbitals of lowest h_pp, in orbital order
    std::vector<int> order(M);
    for (int p = 0; p < M; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(),
                     [&](int p, int q) { return h[(size_t)p * M + p] < h[(size_t)q * M + q]; });
    std::sort(order.begin(), order.begin() + N);
    for (int j = 0; j < N; ++j) U[(size_t)order[j] * N + j] = 1.0;
  }
  std::vector<double> h2((size_t)N * N), e2(n4), Gm(n4), dh((size_t)N * N), deri(n4);
  int done = 0;
  double E_prev = 0.0;
  for (int l = 0; l < o.max_outer; ++l) {
    // integrals in the current orbitals
    HIP_TRY(hipMemcpyAsync(w.U, U.data(), (size_t)M * N * sizeof(double), hipMemcpyHostToDevice, w.s));
    int rc = orb_transform(w);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(e2.data(), w.eri2, n4 * sizeof(double), hipMemcpyDeviceToHost, w.s));
    HIP_TRY(hipStreamSynchronize(w.s));
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        double s = 0.0;
        for (int a = 0; a < M; ++a)
          for (int b = 0; b < M; ++b) s += U[(size_t)a * N + i] * h[(size_t)a * M + b] * U[(size_t)b * N + j];
        h2[(size_t)i * N + j] = s;
      }
    for (int i = 0; i < N; ++i)  // exact symmetry for the solver's 8-fold packing
      for (int j = i + 1; j < N; ++j) {
        const double v = 0.5 * (h2[(size_t)i * N + j] + h2[(size_t)j * N + i]);
        h2[(size_t)i * N + j] = h2[(size_t)j * N + i] = v;
      }
    {
      const size_t n1 = N, n2 = n1 * N, n3 = n2 * N;
      for (size_t p = 0; p < n1; ++p)
        for (size_t q = 0; q <= p; ++q)
          for (size_t r = 0; r < n1; ++r)
            for (size_t s2 = 0; s2 <= r; ++s2) {
              if (p * (p + 1) / 2 + q < r * (r + 1) / 2 + s2) continue;
              const size_t img[8] = {p * n3 + q * n2 + r * n1 + s2, q * n3 + p * n2 + r * n1 + s2,
                                     p * n3 + q * n2 + s2 * n1 + r, q * n3 + p * n2 + s2 * n1 + r,
                                     r * n3 + s2 * n2 + p * n1 + q, s2 * n3 + r * n2 + p * n1 + q,
                                     r * n3 + s2 * n2 + q * n1 + p, s2 * n3 + r * n2 + q * n1 + p};
              double v = 0.0;
              for (size_t m : img) v += e2[m];
              v *= 0.125;
              for (size_t m : img) e2[m] = v;
            }
    }
    // the FCI ground state in them (Alg. 1 or Alg. 2) and its RDMs
    cdfci_opts co;
    memset(&co, 0, sizeof(co));
    co.table_slots = o.table_slots;
    co.z_threshold = o.z_threshold;
    co.dx_threshold = o.cd_dx_threshold;
    co.stream = o.stream;
    cdfci_ctx* ctx = nullptr;
    rc = cdfci_init(h2.data(), e2.data(), N, n_alpha, n_beta, &co, &ctx);
    if (rc) return rc;
    cdfci_stats st;
    rc = cdfci_step(ctx, o.k, o.cd_steps, &st);
    double en[2] = {0.0, 0.0};
    if (!rc) rc = cdfci_rdm_backward(ctx, 1.0, o.top_n, en, dh.data(), deri.data(), nullptr);
    cdfci_free(ctx);
    if (rc) return rc;
    const double E = en[0];
    if (energies) energies[l] = E;
    done = l + 1;
    std::copy(U.begin(), U.end(), U_io);
    if ((l > 0 && std::fabs(E - E_prev) <= o.energy_tol) || l == o.max_outer - 1) break;
    E_prev = E;
    // the orbital problem with the RDMs fixed: gamma = dh, Gamma = 2 deri,
    // symmetrised over the eight permutations that leave (pq|rs) unchanged
    w.g1 = dh;
    const size_t n1 = N, n2 = n1 * N, n3 = n2 * N;
    for (size_t p = 0; p < n1; ++p)
      for (size_t q = 0; q < n1; ++q)
        for (size_t r = 0; r < n1; ++r)
          for (size_t s2 = 0; s2 < n1; ++s2) {
            auto at = [&](size_t a, size_t b, size_t c, size_t d) { return 2.0 * deri[a * n3 + b * n2 + c * n1 + d]; };
            Gm[p * n3 + q * n2 + r * n1 + s2] =
                0.125 * (at(p, q, r, s2) + at(q, p, r, s2) + at(p, q, s2, r) + at(q, p, s2, r) + at(r, s2, p, q) +
                         at(s2, r, p, q) + at(r, s2, q, p) + at(s2, r, q, p));
          }
    HIP_TRY(hipMemcpyAsync(w.Gs, Gm.data(), n4 * sizeof(double), hipMemcpyHostToDevice, w.s));
    std::vector<double> G, Uc = U, Up, Gp, best = U, Un, Gn;
    double val = 0.0;
    rc = orb_eval(w, Uc, &val, G);
    if (rc) return rc;
    double best_val = val;
    for (int k = 0; k < o.max_inner; ++k) {
      if (riemannian_norm(Uc, G, M, N) <= o.grad_tol) break;
      double t = o.step0;
      if (!Up.empty()) {
        std::vector<double> sv(Uc.size()), yv(Uc.size());
        for (size_t q = 0; q < Uc.size(); ++q) {
          sv[q] = Uc[q] - Up[q];
          yv[q] = G[q] - Gp[q];
        }
        const double sy = std::fabs(frob_dot(sv, yv));
        if (sy > 0.0) t = (k % 2 == 1) ? frob_dot(sv, sv) / sy : sy / frob_dot(yv, yv);
      }
      std::vector<double> X(Uc.size());
      for (size_t q = 0; q < Uc.size(); ++q) X[q] = Uc[q] - t * G[q];
      if (!host_orth(X, M, N, Un)) break;
      rc = orb_eval(w, Un, &val, Gn);
      if (rc) return rc;
      Up = Uc;
      Gp = G;
      Uc = Un;
      G = Gn;
      if (val < best_val) {
        best_val = val;
        best = Uc;
      }
    }
    if (p4_values) p4_values[l] = best_val;
    U = best;
  }
  *n_outer = done;
  return 0;
}

// ===========================================================================
// Momentum-space Hubbard model (Sec. 4.1.1 HubbardK) with the
// degenerate-subspace start of Sec. 5.1.3, on the multi-state context.

namespace {

// one-body energies of the Bloch orbitals (row-major momentum index):
// -2t cos(2 pi k_d / n_d) per direction of length n_d >= 3, -t cos(pi k_d)
// for length 2 (one bond, as in the real-space lattice), 0 for length 1
std::vector<double> bloch_levels(const int* dims, int ndim, double t) {
  int L = 1;
  for (int d = 0; d < ndim; ++d) L *= dims[d];
  std::vector<double> eps(L, 0.0);
  for (int k = 0; k < L; ++k) {
    int r = k;
    double e = 0.0;
    for (int d = ndim - 1; d >= 0; --d) {
      const int kd = r % dims[d];
      r /= dims[d];
      if (dims[d] == 2) e += -t * std::cos(M_PI * kd);
      else if (dims[d] >= 3) e += -2.0 * t * std::cos(2.0 * M_PI * kd / dims[d]);
    }
    eps[k] = e;
  }
  return eps;
}

int host_kshift(const int* dims, int ndim, int k, int q, int sgn) {
  int out = 0, mul = 1;
  for (int d = ndim - 1; d >= 0; --d) {
    const int n = dims[d], kd = k % n, qd = q % n;
    k /= n;
    q /= n;
    out += ((kd + sgn * qd + n) % n) * mul;
    mul *= n;
  }
  return out;
}

double host_between_sign(uint64_t s, int x, int y) {
  const int lo = std::min(x, y), hi = std::max(x, y);
  const uint64_t m = ((1ull << hi) - 1ull) & ~((2ull << lo) - 1ull);
  return (__builtin_popcountll(s & m) & 1) ? -1.0 : 1.0;
}

// every string of n electrons with the lowest one-body energy (the Fermi
// shell filled in all ways when it is degenerate)
std::vector<uint64_t> lowest_strings(const std::vector<double>& eps, int n) {
  const int L = (int)eps.size();
  std::vector<int> order(L);
  for (int k = 0; k < L; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return eps[a] < eps[b]; });
  if (n == 0) return {0ull};
  const double ef = eps[order[n - 1]];
  uint64_t base = 0;
  std::vector<int> shell;
  for (int k : order) {
    if (eps[k] < ef - 1e-12) base |= 1ull << k;
    else if (std::fabs(eps[k] - ef) <= 1e-12) shell.push_back(k);
  }
  const int need = n - __builtin_popcountll(base), g = (int)shell.size();
  std::vector<uint64_t> out;
  if (g > 62) return out;
  for (uint64_t m = 0; m < (1ull << g); ++m) {
    if (__builtin_popcountll(m) != need) continue;
    uint64_t s = base;
    for (int i = 0; i < g; ++i)
      if ((m >> i) & 1) s |= 1ull << shell[i];
    out.push_back(s);
  }
  std::sort(out.begin(), out.end());
  return out;
}

constexpr int kMaxBlock = 2048;

int x_setup_k(cdfci_xctx* X, const int* dims, int ndim, double t, double U) {
  cdfci_ctx* c = X->base;
  const int L = c->N, na = c->na, nb = c->nb, n = X->n;
  const std::vector<double> eps = bloch_levels(dims, ndim, t);
  HIP_TRY(hipMalloc(&X->d_eps, L * sizeof(double)));
  HIP_TRY(hipMemcpy(X->d_eps, eps.data(), L * sizeof(double), hipMemcpyHostToDevice));
  X->hk.L = L;
  X->hk.ndim = ndim;
  for (int d = 0; d < 3; ++d) X->hk.dims[d] = d < ndim ? dims[d] : 1;
  X->hk.eps = X->d_eps;
  X->hk.u = U / L;
  int rc = x_alloc(X);
  if (rc) return rc;
  // the degenerate block and H - shift on it
  const std::vector<uint64_t> sa = lowest_strings(eps, na), sb = lowest_strings(eps, nb);
  const size_t m = sa.size() * sb.size();
  if (m < (size_t)n || m > (size_t)kMaxBlock) return CDFCI_ERR_UNSUPPORTED;
  std::vector<std::pair<uint64_t, uint64_t>> keys;
  for (uint64_t a : sa)
    for (uint64_t b : sb) keys.push_back({a, b});
  std::vector<double> Hs(m * m, 0.0);
  for (size_t j = 0; j < m; ++j) {
    const uint64_t a = keys[j].first, b = keys[j].second;
    double d = X->hk.u * na * nb - X->shift;
    for (int k = 0; k < L; ++k) d += eps[k] * (double)(((a >> k) & 1) + ((b >> k) & 1));
    Hs[j * m + j] = d;
    for (int k = 0; k < L; ++k) {
      if (!((a >> k) & 1)) continue;
      for (int p = 0; p < L; ++p) {
        if (!((b >> p) & 1)) continue;
        for (int q = 1; q < L; ++q) {
          const int kq = host_kshift(dims, ndim, k, q, 1), pq = host_kshift(dims, ndim, p, q, -1);
          if (((a >> kq) & 1) || ((b >> pq) & 1)) continue;
          const uint64_t a2 = a ^ (1ull << k) ^ (1ull << kq), b2 = b ^ (1ull << p) ^ (1ull << pq);
          const auto it = std::lower_bound(keys.begin(), keys.end(), std::make_pair(a2, b2));
          if (it == keys.end() || *it != std::make_pair(a2, b2)) continue;
          Hs[(size_t)(it - keys.begin()) * m + j] +=
              X->hk.u * host_between_sign(a, k, kq) * host_between_sign(b, p, pq);
        }
      }
    }
  }
  std::vector<double> w, V;
  host_sym_eig(Hs, (int)m, w, V);
  std::vector<int> ord(m);
  for (size_t i = 0; i < m; ++i) ord[i] = (int)i;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return w[x] < w[y]; });
  std::vector<double> coef(m * n);
  std::vector<XInitTask> tasks(m);
  for (size_t i = 0; i < m; ++i) tasks[i] = XInitTask{keys[i].first, keys[i].second};
  for (int k = 0; k < n; ++k) {
    const int col = ord[k];
    if (!(w[col] < 0.0)) return CDFCI_ERR_NOT_NEGATIVE;
    size_t big = 0;
    for (size_t i = 1; i < m; ++i)
      if (std::fabs(V[i * m + col]) > std::fabs(V[big * m + col])) big = i;
    const double scale = std::sqrt(-w[col]) * (V[big * m + col] < 0.0 ? -1.0 : 1.0);
    for (size_t i = 0; i < m; ++i) coef[i * n + k] = scale * V[i * m + col];
  }
  hipStream_t s = c->stream;
  CallBufs bufs;
  XInitTask* d_tasks;
  double* d_coef;
  HIP_TRY(bufs.alloc(&d_tasks, m));
  HIP_TRY(bufs.alloc(&d_coef, m * n));
  HIP_TRY(hipMemcpyAsync(d_tasks, tasks.data(), m * sizeof(XInitTask), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_coef, coef.data(), m * n * sizeof(double), hipMemcpyHostToDevice, s));
  k_xinit_insert<<<(unsigned)((m + 63) / 64), 64, 0, s>>>(X->K, X->R, X->mask, d_tasks, d_coef, (int)m, n, X->x);
  const int chunks = (int)std::min<int64_t>((X->n_col + 255) / 256, 64);
  k_xinit_scatter_k<<<dim3(chunks, (unsigned)m), 256, 0, s>>>(X->hk, X->K, X->R, X->mask, d_tasks, d_coef, n, na,
                                                                nb, X->shift, X->x);
  k_xinit_matrices<<<1, 1, 0, s>>>(X->K, X->R, X->mask, d_tasks, (int)m, n, X->x);
  HIP_TRY(hipGetLastError());
  rc = x_first(X);
  HIP_TRY(hipStreamSynchronize(s));
  return rc;
}

}  // namespace

extern "C" int cdfci_xinit_hubbard_k(const int* dims, int ndim, double t, double U, int n_alpha, int n_beta,
                                     int n_states, double shift, const cdfci_opts* opts, cdfci_xctx** out) {
  if (!dims || ndim < 1 || ndim > 3 || !out) return CDFCI_ERR_INVALID_ARG;
  int L = 1;
  for (int i = 0; i < ndim; ++i) {
    if (dims[i] < 1) return CDFCI_ERR_INVALID_ARG;
    L *= dims[i];
  }
  if (L > kMaxOrb) return CDFCI_ERR_UNSUPPORTED;
  if (L < 2 || !std::isfinite(t) || !std::isfinite(U)) return CDFCI_ERR_INVALID_ARG;
  cdfci_xctx* X = nullptr;
  int rc = x_create(L, n_alpha, n_beta, n_states, shift, opts, out, &X);
  if (rc) return rc;
  X->kind = 1;
  rc = x_setup_k(X, dims, ndim, t, U);
  if (rc) {
    cdfci_xfree(X);
    return rc;
  }
  *out = X;
  return 0;
}
