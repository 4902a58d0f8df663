// Batched single-coordinate descent (Alg. 1) on many periodic Hubbard
// lattices (Sec. 2.2) in one persistent kernel.  Included into cdfci.hip
// inside its kernel namespace.
//
// A Hubbard column holds the diagonal U * (doubly occupied sites) and one hop
// per (bond, spin) whose two sites differ in occupation, at most 1 + 2 * bonds
// entries (65 on a 4x4 lattice), so one wavefront owns one instance and runs
// a whole step with no device-wide synchronisation: lane l takes hop slots
// l, l + 64, ... (slot = 2 * bond + spin).  Each instance keeps its own hash
// table, which only the wave holding the instance touches, so b updates are
// plain stores; lanes claim empty slots with a CAS, one probe round at a time,
// so two lanes of the wave never wait on each other.  Waves take instances
// from a queue and run up to `chunk` steps on each before taking the next.

constexpr int kHubMaxBonds = 64;

struct HubInst {
  Slot* T;
  uint64_t mask, max_entries;
  Ctl* ctl;                 // the instance's scalar state (as the single-instance path keeps it)
  int64_t step_limit;       // run until ctl->steps reaches this
  unsigned long long* elements;  // column entries enumerated (device counter)
  double t, U;
  int nbonds, pad;
  uint8_t bi[kHubMaxBonds], bj[kHubMaxBonds];
};

struct HubArgs {
  const HubInst* inst;    // every instance of the batch
  const unsigned* active; // ids of the resident instances this launch serves
  int n_inst;             // entries of `active`
  unsigned* queue;  // [0] next instance, [1] instances still running after their visit
  int64_t chunk;
  double tau, theta, dx_tol;
  int trace_inst;   // instance whose steps are recorded (-1: none)
  double* tr_E;
  uint64_t *tr_a, *tr_b;
};

// Values every lane holds identically, moved to scalar registers.  All
// branches that steer the instance and step loops test such values, so the
// compiler sees wave-uniform control flow and never splits the wave's lanes
// across loop iterations (the shuffles and ballots need all 64 lanes).
__device__ __forceinline__ uint32_t uni32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni32((uint32_t)(v >> 32)) << 32) | uni32((uint32_t)v);
}
__device__ __forceinline__ double unid(double v) {
  return __longlong_as_double((long long)uni64((uint64_t)__double_as_longlong(v)));
}

// wave-wide sum in a fixed pairing order (every lane gets the same value)
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off);
    v = (threadIdx.x & off) ? (o + v) : (v + o);
  }
  return v;
}

__device__ __forceinline__ void wave_best(Cand& best) {
  for (int off = 32; off > 0; off >>= 1) {
    const Cand o = shfl_cand(best, (threadIdx.x & 63) ^ off);
    if (better(o, best)) best = o;
  }
}

__global__ void k_hub_reset(unsigned* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    queue[0] = 0u;
    queue[1] = 0u;
  }
}

__global__ void __launch_bounds__(64) k_hub_batch(HubArgs A) {
  const int lane = threadIdx.x;
  // No branch below depends on the lane index: lane-0-only work is written as
  // work every lane does with identical values (or an increment of 0), so the
  // wave stays whole on every path.
  for (;;) {
    const unsigned got = atomicAdd(&A.queue[0], lane == 0 ? 1u : 0u);
    const unsigned q = uni32(got);
    if (q >= (unsigned)A.n_inst) break;
    const unsigned id = uni32(A.active[q]);
    const HubInst& P = A.inst[id];
    Slot* T = P.T;
    const uint64_t mask = uni64(P.mask);
    Ctl* ctl = P.ctl;
    const int64_t step0 = (int64_t)uni64((uint64_t)ctl->steps);
    const int64_t limit = (int64_t)uni64((uint64_t)P.step_limit);
    const int skip = (int)uni32((uint32_t)(ctl->error | ctl->stopped));
    const int64_t todo = skip ? 0 : (limit - step0 < A.chunk ? limit - step0 : A.chunk);
    if (todo > 0) {
    const double t = unid(P.t), U = unid(P.U);
    const int nslot = 2 * (int)uni32((uint32_t)P.nbonds);
    dd mu{unid(ctl->mu_hi), unid(ctl->mu_lo)}, al{unid(ctl->al_hi), unid(ctl->al_lo)};
    double d = unid(ctl->d);
    uint64_t sa = uni64(ctl->sel_a), sb = uni64(ctl->sel_b);
    int64_t sslot = (int64_t)uni64((uint64_t)ctl->sel_slot);
    double sc = unid(ctl->sel_c), sbv = unid(ctl->sel_b_val);
    unsigned long long occupied = ctl->occupied, inserts = 0, elements = 0;
    int max_probe = ctl->max_probe;
    int flags = 0, stopped = 0;
    const bool trace = (int)id == A.trace_inst;
    int64_t step = 0;
    for (; step < todo; ++step) {
      const double Hii = U * (double)__popcll(sa & sb);
      const double mud = dd_val(mu);
      const double eta = unid(line_search(4.0 * sbv + 4.0 * mud * sc, 2.0 * Hii + 4.0 * sc * sc + 2.0 * mud,
                                          4.0 * sc));
      // mu += 2 eta c_i + eta^2 ; alpha += 2 eta b_i + eta^2 H_ii (pre-step c_i, b_i)
      const dd e2 = two_prod(eta, eta);
      mu = dd_add(dd_add(mu, two_prod(2.0 * eta, sc)), e2);
      al = dd_add(dd_add(al, two_prod(2.0 * eta, sbv)), dd_mul_d(e2, Hii));
      const double mu1 = dd_val(mu);
      const double cnew = sc + eta;
      Cand best{-1.0, kEmpty, kEmpty, -1, 0.0, 0.0};
      double rs = 0.0;
      int n_ins = 0, n_valid = 0, lflags = 0, lprobe = 0;
      for (int base = 0; base < nslot; base += 64) {
        const int s = base + lane;
        bool valid = false;
        uint64_t ja = sa, jb = sb;
        double Hj = 0.0;
        if (s < nslot) {
          const int e = s >> 1, spin = s & 1;
          const int i = P.bi[e], j = P.bj[e];
          const uint64_t str = spin ? sb : sa;
          const int oi = (int)((str >> i) & 1), oj = (int)((str >> j) & 1);
          if (oi != oj) {
            const int lo = min(i, j), hi = max(i, j);
            // electrons of this spin strictly between the two sites
            const uint64_t between = ((1ull << hi) - 1ull) & ~((2ull << lo) - 1ull);
            const int neg = __popcll(str & between) & 1;
            Hj = neg ? t : -t;
            const uint64_t ns = str ^ ((1ull << i) | (1ull << j));
            if (spin) jb = ns;
            else ja = ns;
            valid = Hj != 0.0;
          }
        }
        // find
        int64_t slot = -1;
        double cj = 0.0, bj = 0.0;
        uint64_t idx = 0;
        int probes = 0;
        if (valid) {
          idx = hash_key(ja, jb) & mask;
          for (; probes < kMaxProbe; ++probes) {
            const uint64_t ka = ld_co(&T[idx].ka);
            if (ka == kEmpty) break;
            if (ka == ja && ld_co(&T[idx].kb) == jb) {
              slot = (int64_t)idx;
              cj = ld_co(&T[idx].c);
              bj = ld_co(&T[idx].b);
              break;
            }
            idx = (idx + 1) & mask;
          }
          if (probes >= kMaxProbe) lflags |= kErrTableFull;
        }
        const double delta = eta * Hj;
        double bnew = 0.0;
        if (slot >= 0) {
          bnew = bj;
          if (cj != 0.0 || fabs(delta) >= A.tau) {
            bnew = bj + delta;
            st_co(&T[slot].b, bnew);
          }
        }
        // insert: claim the first empty slot of the probe sequence, one round
        // per collision with another lane of this wave
        bool need = valid && slot < 0 && probes < kMaxProbe && fabs(delta) >= A.tau;
        while (__ballot(need)) {
          if (need) {
            const unsigned long long old =
                atomicCAS((unsigned long long*)&T[idx].ka, (unsigned long long)kEmpty, (unsigned long long)ja);
            if (old == (unsigned long long)kEmpty) {
              st_co(&T[idx].kb, jb);
              st_co(&T[idx].c, 0.0);
              st_co(&T[idx].b, delta);
              slot = (int64_t)idx;
              bnew = delta;
              need = false;
              ++n_ins;
            } else {
              idx = (idx + 1) & mask;
              if (++probes >= kMaxProbe) {
                need = false;
                lflags |= kErrTableFull;
              }
            }
          }
        }
        if (valid) {
          ++n_valid;
          rs += Hj * cj;
          lprobe = max(lprobe, probes + 1);
          // entries not stored (compressed away) are not candidates
          if (slot >= 0) {
            const Cand c{fabs(4.0 * bnew + 4.0 * mu1 * cj), ja, jb, slot, bnew, cj};
            if (better(c, best)) best = c;
          }
        }
      }
      rs = wave_sum(rs);
      wave_best(best);
      for (int off = 32; off > 0; off >>= 1) {
        n_ins += __shfl_xor(n_ins, off);
        n_valid += __shfl_xor(n_valid, off);
        lflags |= __shfl_xor(lflags, off);
        lprobe = max(lprobe, __shfl_xor(lprobe, off));
      }
      rs = unid(rs);
      n_ins = (int)uni32((uint32_t)n_ins);
      n_valid = (int)uni32((uint32_t)n_valid);
      flags |= (int)uni32((uint32_t)lflags);
      lprobe = (int)uni32((uint32_t)lprobe);
      max_probe = max(max_probe, lprobe);
      occupied += (unsigned long long)n_ins;
      inserts += (unsigned long long)n_ins;
      elements += (unsigned long long)(n_valid + 1);
      if (occupied > P.max_entries) flags |= kErrTableFull;
      const double R = Hii * cnew + rs;
      st_co(&T[sslot].c, cnew);
      st_co(&T[sslot].b, R);
      if (trace) {
        A.tr_E[step0 + step] = dd_val(al) / mu1;
        A.tr_a[step0 + step] = sa;
        A.tr_b[step0 + step] = sb;
      }
      const Cand self{fabs(4.0 * R + 4.0 * mu1 * cnew), sa, sb, sslot, R, cnew};
      if (better(self, best)) best = self;
      d = (step0 + step == 0) ? fabs(eta) : A.theta * d + (1.0 - A.theta) * fabs(eta);
      sa = uni64(best.a);
      sb = uni64(best.b);
      sslot = (int64_t)uni64((uint64_t)best.slot);
      sc = unid(best.c);
      sbv = unid(best.bnew);
      // this wave's stores complete before the next step's probes read them
      __builtin_amdgcn_s_waitcnt(0);
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
    // write-back: every lane stores the same values
    const unsigned long long ins0 = ctl->inserts, el0 = *P.elements;
    const int err0 = ctl->error;
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
    ctl->steps = step0 + step;
    ctl->occupied = occupied;
    ctl->inserts = ins0 + inserts;
    ctl->max_probe = max_probe;
    ctl->error = err0 | flags;
    ctl->stopped = stopped;
    *P.elements = el0 + elements;
    if (!stopped && !flags && step0 + step < limit) atomicAdd(&A.queue[1], lane == 0 ? 1u : 0u);
    }
  }
}
