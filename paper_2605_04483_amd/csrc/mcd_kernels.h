// Multicoordinate descent, mCDFCI (paper Sec. 3.2, Algorithm 2), device side.
// Included into cdfci.hip inside its kernel namespace (uses Ctl, Cand, Slot).
//
// One step is a fixed sequence of launches with no host synchronisation:
//   select   top-k of |4 b_j + 4 mu c_j| over the step's candidates (the union
//            of the previous step's columns, each determinant once): every
//            candidate position's key, a bound below which fewer than k
//            distinct determinants cannot lie, repeats dropped above it, then
//            an MSB radix select on the bit pattern of the non-negative double
//            |g| (in one workgroup, or grid passes for large k), exact ties at
//            the threshold to the smaller key;
//   H_II     pairwise Slater-Condon entries among the chosen determinants;
//   reduced  A = Q^T H Q with Q = [c~, E_I] (eq. (def-z)); its lowest
//            eigenpair by LOBPCG started from the current point [nu; c_I];
//            gamma, eta; mu and alpha.  The same launch's other workgroups
//            run the probe half of the scatter, which needs the chosen set but
//            not eta: the k columns enumerated, their entries looked up once,
//            each entry's slot written at its own candidate position,
//            recalculation sums for b_I, one record per entry;
//   apply    b += H_{:,I} eta from the records with the compression rule
//            (inserting the absent entries whose increment is kept);
//   finish   b_I <- recalculated values, I appended to the candidates.
// c and b are stored with a lazy global scale: c = s * c_hat, b = s * b_hat, so
// the gamma rescaling of every entry costs one scalar update (s <- gamma s).
//
// Candidates live in pages of 256 slot ids with a count per page.  Each
// scatter workgroup owns one page, so no global append counter is contended.

struct McState {
  unsigned long long n_pages;        // candidate pages of the coming selection
  unsigned long long prefix, pmask;  // radix select: fixed bits and their mask
  long long need;                    // still to take inside the current bucket
  unsigned long long n_above;        // strictly above the bucket (selected)
  unsigned long long n_sel, n_tie;   // gather counters
  unsigned long long n_dense;        // entries of a dense candidate list (mode entry)
  int all, done;                     // all candidates selected / bucket exact
  double scale;                      // s in c = s * c_hat
  double inv_scale;                  // 1 / s after this step's update
  double gamma;
  int eig_iters;                     // iterations of the last reduced problem
  int rescale;
  int skip;  // this step does nothing (an error is pending or the run stopped)
  unsigned arrive;                   // workgroups done with the current selection kernel
  unsigned long long n_total;        // candidates of the coming selection
  unsigned long long last_sel;       // size of the last completed step's chosen set
  unsigned long long lowkey;         // keys >= lowkey take the exact (de-duplicating) pass
  int pred_d;                        // top digit of the last step's boundary (-1: none)
  // running totals of the selections (inspection): selections, candidate
  // positions holding a slot, slots kept by the exact pass, bound failures
  unsigned long long acc_sel, acc_pos, acc_kept, acc_fallback;
  unsigned arrive_cols;              // workgroups of k_mc_colfinish done (the last one resets it)
};

constexpr int kPage = 256;
// A candidate position that holds no slot (the entry is absent, zero, or in
// the chosen set), and the selection key of a position that holds none; a key
// of a real candidate is the bit pattern of a non-negative double, so bit 63
// is free.
constexpr unsigned kNoCand = 0xffffffffu;
constexpr unsigned long long kKeyExcluded = 1ull << 63;
constexpr int kRadixBits = 11;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixPasses = 6;  // digits at bits 53, 42, 31, 20, 9 (11 wide) and 0 (9 wide)
constexpr int kMaxTies = 4096;
constexpr int kSelBlocks = 1024;  // workgroups of the selection launches
// nu^2 = ||c - E_I c_I||^2 is formed as mu - c_I.c_I.  mu is carried from
// step to step while the stored c is rounded at every update, so the two
// drift apart by a few ulps of mu per step; below this fraction of mu nu^2
// cannot be told from that drift and the c~ column is dropped (nu = 0,
// gamma = 1).  A genuine nu^2 this small changes the step's energy by about
// the same relative amount.
constexpr double kNu2Floor = 0x1p-36;

__device__ __forceinline__ int radix_shift(int pass) { return pass < 5 ? 53 - 11 * pass : 0; }
__device__ __forceinline__ unsigned long long radix_digit_mask(int pass) {
  return pass < 5 ? 0x7FFull : 0x1FFull;
}

__device__ __forceinline__ unsigned long long g_key_cb(double c, double b, double mu) {
  double g = fabs(4.0 * b + 4.0 * mu * c);
  return (unsigned long long)__double_as_longlong(g);
}
__device__ __forceinline__ unsigned long long g_key(const Slot& s, double mu) { return g_key_cb(s.c, s.b, mu); }

// |c| as an ordered key (selection of the largest coefficients)
__device__ __forceinline__ unsigned long long c_key(const Slot& s) {
  return (unsigned long long)__double_as_longlong(fabs(s.c));
}

// all occupied slots become candidates (entering the multicoordinate mode):
// a dense list, turned into full pages by k_mc_dense_pages
__global__ void __launch_bounds__(256) k_mc_init_cands(const Slot* T, uint64_t nslots,
                                                       unsigned* cand, McState* st, uint64_t cap) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (T[i].ka == kEmpty) continue;
    unsigned long long k = atomicAdd(&st->n_dense, 1ull);
    if (k < cap) cand[k] = (unsigned)i;
  }
}

__global__ void __launch_bounds__(256) k_mc_dense_pages(unsigned* cnt, McState* st, uint64_t cap) {
  const unsigned long long n = min(st->n_dense, (unsigned long long)cap);
  const unsigned long long pages = (n + kPage - 1) / kPage;
  for (unsigned long long p = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; p < pages;
       p += (unsigned long long)gridDim.x * blockDim.x)
    cnt[p] = (unsigned)min((unsigned long long)kPage, n - p * kPage);
  // every workgroup reads n_dense above, so it is reset by k_mc_clear (which
  // runs before the next list is built), not here
  if (blockIdx.x == 0 && threadIdx.x == 0) st->n_pages = pages;
}

// clear the candidate bitmap and the gather counters (entering the
// multicoordinate state; inside a step k_mc_tail clears the words it used)
__global__ void __launch_bounds__(256) k_mc_clear(unsigned* bitmap, uint64_t nwords, McState* st) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
       i += (uint64_t)gridDim.x * blockDim.x)
    bitmap[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->n_tie = 0;
    st->n_dense = 0;
  }
}

__global__ void __launch_bounds__(256) k_mc_clear_words(unsigned* bitmap, uint64_t nwords) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
       i += (uint64_t)gridDim.x * blockDim.x)
    bitmap[i] = 0u;
}

// ---------------------------------------------------------------- selection with last-workgroup scans

// Radix-select state as kept by McState between the selection kernels.
struct SelState {
  unsigned long long prefix, pmask, n_above;
  long long need;
  int all, done;
};

// True in the one workgroup that finishes a launch last.  Everything the
// workgroups share is written with agent-scope atomics, which are performed
// at the coherence point, so a workgroup only has to wait for its own memory
// operations to complete before it arrives (no cache write-back: a fence at
// agent scope would write back the XCD's whole L2), and the last one reads
// with agent-scope loads.
__device__ bool last_workgroup(unsigned* arrive) {
  __shared__ int s_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  return s_last != 0;
}

// The last workgroup of a histogram pass (256 threads): choose the radix
// digit of the bucket holding the k-th largest key from the global
// histogram (read with agent-scope loads), advance the state in McState, and
// clear the histogram and the arrival count for the next pass.  Suffix counts
// come from a block scan (per-wave shuffles, then the wave totals), so no
// thread walks more than its own eight bins.
__device__ void mc_scan_last(unsigned* hist, McState* st, int k, int pass) {
  __shared__ SelState S;
  __shared__ unsigned long long s_wt[4];
  __shared__ int s_d;
  __shared__ unsigned long long s_above;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) {
    if (pass == 0) {
      const unsigned long long total =
          __hip_atomic_load(&st->n_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      S.prefix = 0;
      S.pmask = 0;
      S.n_above = 0;
      S.done = 0;
      S.all = (total <= (unsigned long long)k) ? 1 : 0;
      S.need = k;
    } else {
      S.prefix = st->prefix;
      S.pmask = st->pmask;
      S.n_above = st->n_above;
      S.need = st->need;
      S.all = st->all;
      S.done = st->done;
    }
  }
  __syncthreads();
  if (!(S.all || S.done)) {
    const int sh = radix_shift(pass);
    const int nb = (int)radix_digit_mask(pass) + 1;
    const int per = nb / 256;  // 8 (11-bit digits) or 2 (the last, 9-bit digit)
    const int lo = tid * per;
    unsigned hv[8];
    unsigned long long run = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      hv[u] = u < per ? __hip_atomic_load(&hist[lo + u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
      run += hv[u];
    }
    // inclusive suffix over the wave's lanes, then over the waves
    unsigned long long x = run;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long y = __shfl_down(x, o);
      if (lane + o < 64) x += y;
    }
    if (lane == 0) s_wt[w] = x;
    if (tid == 0) s_d = -1;
    __syncthreads();
    unsigned long long acc = x - run;  // keys in bins above this thread's, within the wave
    for (int q = w + 1; q < 4; ++q) acc += s_wt[q];
    const long long need = S.need;
    unsigned hd_mine = 0;
    for (int u = per - 1; u >= 0; --u) {
      const long long above = (long long)acc;
      if (above < need && above + (long long)hv[u] >= need) {
        s_d = lo + u;
        s_above = acc;
        hd_mine = hv[u];
      }
      acc += hv[u];
    }
    __syncthreads();
    if (s_d >= 0 && tid == s_d / per) {  // the thread that owns the chosen bin
      const long long above = (long long)s_above;
      S.n_above += (unsigned long long)above;
      S.need = need - above;
      S.prefix |= (unsigned long long)s_d << sh;
      S.pmask |= radix_digit_mask(pass) << sh;
      if ((long long)hd_mine == need - above) S.done = 1;
    }
  }
  __syncthreads();
  if (tid == 0) {  // read by the following launches
    st->prefix = S.prefix;
    st->pmask = S.pmask;
    st->n_above = S.n_above;
    st->need = S.need;
    st->all = S.all;
    st->done = S.done;
    st->arrive = 0;
  }
  for (int i = tid; i < kRadixBins; i += blockDim.x) hist[i] = 0u;
}

// The selection's dense lists: pass 0 writes the kept candidates of
// workgroup b (key and slot) to region b, whose length it records in
// count[b]; the later passes and the gather read only those.  A region holds
// as many entries as the positions its workgroup visits, so the arrays need
// the positions plus one grid of slack.
struct SelBufs {
  unsigned long long* key;
  unsigned* slot;
  unsigned* count;  // kSelBlocks
};

__device__ __forceinline__ unsigned long long sel_region(unsigned long long n) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  return (n + stride - 1) / stride * blockDim.x;
}

// One radix-select pass over the step's candidates; pass 0 also computes the
// keys (|g|, or |c| when by_c is set), counts the candidates and compacts
// them into the dense lists, taking every position as a distinct candidate
// (the selection of the largest |c| of the reverse pass).  The last
// workgroup to finish chooses the digit.
__global__ void __launch_bounds__(256) k_mc_radix(const Slot* T, const unsigned* cand, const unsigned* cnt,
                                                  SelBufs D, const Ctl* ctl, McState* st, unsigned* hist,
                                                  int pass, int by_c, int k) {
  __shared__ unsigned h[kRadixBins];
  __shared__ unsigned s_wn[4];
  __shared__ unsigned s_run;
  if (st->skip) return;
  if (pass > 0 && (st->all || st->done)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < kRadixBins; i += blockDim.x) h[i] = 0u;
  if (tid == 0) s_run = 0u;
  __syncthreads();
  const unsigned long long n = st->n_pages * kPage;
  const unsigned long long region = sel_region(n), base = blockIdx.x * region;
  const double mu = ctl->mu_hi + ctl->mu_lo;
  const int sh = radix_shift(pass);
  const unsigned long long dm = radix_digit_mask(pass);
  const unsigned long long P = st->prefix, M = st->pmask;
  if (pass == 0) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i0 = (unsigned long long)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
      const unsigned long long i = i0 + tid;
      bool keep = false;
      unsigned sl = 0u;
      unsigned long long key = 0ull;
      if (i < n && (i & (kPage - 1)) < cnt[i / kPage]) {
        sl = cand[i];
        keep = sl != kNoCand;
        if (keep) {
          key = by_c ? c_key(T[sl]) : g_key(T[sl], mu);
          atomicAdd(&h[(key >> sh) & dm], 1u);
        }
      }
      const unsigned long long bal = __ballot(keep);
      if (lane == 0) s_wn[w] = (unsigned)__popcll(bal);
      __syncthreads();
      unsigned off = s_run;
      for (int q = 0; q < w; ++q) off += s_wn[q];
      if (keep) {
        const unsigned long long at = base + off + (unsigned)__popcll(bal & ((1ull << lane) - 1ull));
        D.key[at] = key;
        D.slot[at] = sl;
      }
      __syncthreads();
      if (tid == 0) s_run += s_wn[0] + s_wn[1] + s_wn[2] + s_wn[3];
    }
    __syncthreads();
  } else {
    const unsigned nb = D.count[blockIdx.x];
    for (unsigned j = tid; j < nb; j += blockDim.x) {
      const unsigned long long key = D.key[base + j];
      if ((key & M) != P) continue;
      atomicAdd(&h[(key >> sh) & dm], 1u);
    }
    __syncthreads();
  }
  for (int i = tid; i < kRadixBins; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
  if (pass == 0 && tid == 0) {
    D.count[blockIdx.x] = s_run;
    if (s_run) atomicAdd(&st->n_total, (unsigned long long)s_run);
  }
  if (last_workgroup(&st->arrive)) mc_scan_last(hist, st, k, pass);
}

// ---------------------------------------------------------------- keys first, then the exact pass near the top
//
// A slot reached from several chosen columns sits at several positions of the
// candidate list with one key, and Alg. 2 ranks it once.  Dropping the repeats
// costs a returning atomic per position, so it is done only where the ranking
// is decided.  A column holds a determinant at most once, so a slot sits at
// most last_sel + 1 times in the list (once per previous column and once in
// the chosen set's own page; once when the list was built from the table):
// the R = k (last_sel + 1) largest position keys hold at least k distinct
// slots (when all positions are fewer than R, every one is ranked).  k_mc_keys forms every position's key (one random read of the
// slot's c and b), counts the positions per top digit, repeats included, and
// finds the digit d holding the R-th largest.  The bin of one top digit spans
// two binades and can hold most of the positions, so k_mc_keys also counts
// the positions of the previous step's boundary digit per second digit: when
// the boundary stays in that bin (the usual case) the second digit holding
// the R-th largest narrows the bound to 2^-10 of a binade.  The bound is the
// key lowkey (d, or d and the second digit, followed by zeros); k_mc_dedup
// keeps the first position of each slot among the keys >= lowkey, counting
// them exactly, and the ranking of the lower keys is not needed (every slot
// above them is kept).  k_mc_tail checks the count: fewer than k distinct
// slots above a nonzero bound would mean the bound failed, and the step then
// stops with kErrSelect instead of choosing from an incomplete set.

// The last workgroup (256 threads) of a histogram launch: the digit holding
// the need-th largest key of a 2048-bin histogram (counted from the top), or
// -1 when it holds fewer keys; *above = the keys in the bins above it and
// *total = all of its keys.  Thread t reads bins 8t..8t+7 with agent-scope
// loads.
__device__ int digit_of_rank(const unsigned* hist, long long need, unsigned long long* above,
                             unsigned long long* total) {
  __shared__ unsigned long long s_wt[4];
  __shared__ unsigned long long s_above;
  __shared__ int s_d;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  unsigned hv[8];
  unsigned long long run = 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    hv[u] = __hip_atomic_load(&hist[tid * 8 + u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    run += hv[u];
  }
  unsigned long long x = run;  // inclusive suffix over the wave's lanes
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_down(x, o);
    if (lane + o < 64) x += y;
  }
  if (lane == 0) s_wt[w] = x;
  if (tid == 0) s_d = -1;
  __syncthreads();
  unsigned long long acc = x - run;
  for (int q = w + 1; q < 4; ++q) acc += s_wt[q];
  for (int u = 7; u >= 0; --u) {
    if ((long long)acc < need && (long long)(acc + hv[u]) >= need) {
      s_d = tid * 8 + u;
      s_above = acc;
    }
    acc += hv[u];
  }
  __syncthreads();
  *above = s_d >= 0 ? s_above : 0ull;
  *total = s_wt[0] + s_wt[1] + s_wt[2] + s_wt[3];
  return s_d;
}

// The first kernel of a step: nothing runs when an error is pending or the
// stopping rule fired (k_mc_bound records the same test as st->skip for the
// rest of the step).
__device__ __forceinline__ bool step_off(const Ctl* ctl) { return ctl->error || ctl->stopped; }

// pkey[i] = the key of the slot at candidate position i (kKeyExcluded where
// there is none); hist counts every position per top digit and hist2 the
// positions of top digit pred_d per second digit.  Each thread takes four
// positions a round so that four slot reads are in flight.  The keys are
// formed from the stored c^, b^ (the lazy scale multiplies every key alike).
__global__ void __launch_bounds__(256) k_mc_keys(const Slot* T, const unsigned* cand, const unsigned* cnt,
                                                 unsigned long long* pkey, const Ctl* ctl, const McState* st,
                                                 unsigned* hist, unsigned* hist2) {
  constexpr int U = 4;
  __shared__ unsigned h[kRadixBins], h2[kRadixBins];
  if (step_off(ctl)) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < kRadixBins; i += blockDim.x) {
    h[i] = 0u;
    h2[i] = 0u;
  }
  const unsigned long long pd = (unsigned long long)st->pred_d;  // all ones when there is none
  __syncthreads();
  const unsigned long long n = st->n_pages * kPage;
  const double mu = ctl->mu_hi + ctl->mu_lo;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x * U;
  for (unsigned long long i0 = (unsigned long long)blockIdx.x * blockDim.x * U + tid; i0 < n; i0 += stride) {
    unsigned sl[U];
    double2 cb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned long long i = i0 + (unsigned long long)u * blockDim.x;
      sl[u] = (i < n && (i & (kPage - 1)) < cnt[i / kPage]) ? cand[i] : kNoCand;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      cb[u] = sl[u] != kNoCand ? *reinterpret_cast<const double2*>(&T[sl[u]].c) : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned long long i = i0 + (unsigned long long)u * blockDim.x;
      if (i >= n) continue;
      unsigned long long key = kKeyExcluded;
      if (sl[u] != kNoCand) {
        key = g_key_cb(cb[u].x, cb[u].y, mu);
        const unsigned long long d = key >> radix_shift(0);
        atomicAdd(&h[d], 1u);
        if (d == pd) atomicAdd(&h2[(key >> radix_shift(1)) & radix_digit_mask(1)], 1u);
      }
      pkey[i] = key;
    }
  }
  __syncthreads();
  for (int i = tid; i < kRadixBins; i += blockDim.x) {
    if (h[i]) atomicAdd(&hist[i], h[i]);
    if (h2[i]) atomicAdd(&hist2[i], h2[i]);
  }
}

// One workgroup of 256 threads after k_mc_keys: the start of the step (the
// previous step's scale fold has completed; counters reset; st->skip), then
// lowkey (0 when there are at most R positions) and pred_d from the two
// histograms, which it clears.
__global__ void __launch_bounds__(256) k_mc_bound(McState* st, const Ctl* ctl, unsigned* hist, unsigned* hist2,
                                                  int k) {
  const int tid = threadIdx.x;
  const bool off = step_off(ctl);
  if (tid == 0) {
    if (st->rescale) {
      st->scale = 1.0;
      st->inv_scale = 1.0;
      st->rescale = 0;
    }
    st->arrive = 0;
    st->n_total = 0;
    st->skip = off ? 1 : 0;
  }
  if (off) return;  // k_mc_keys did not run: the histograms are clear
  const long long rank = (long long)k * (long long)(st->last_sel + 1);  // last_sel <= 1024
  const unsigned long long pd = (unsigned long long)st->pred_d;
  unsigned long long above = 0, total = 0;
  const int d = digit_of_rank(hist, rank, &above, &total);  // -1: at most rank positions in all
  int d2 = -1;
  if (d >= 0 && (unsigned long long)d == pd) {  // uniform: d and pd are the same in every thread
    unsigned long long above2 = 0, total2 = 0;
    d2 = digit_of_rank(hist2, rank - (long long)above, &above2, &total2);
  }
  if (tid == 0) {
    st->acc_pos += total;
    unsigned long long lk = 0ull;
    if (d >= 0) lk = (unsigned long long)d << radix_shift(0);
    if (d2 >= 0) lk |= (unsigned long long)d2 << radix_shift(1);
    st->lowkey = lk;
    if (d >= 0) st->pred_d = d;
  }
  for (int i = tid; i < kRadixBins; i += blockDim.x) {
    hist[i] = 0u;
    hist2[i] = 0u;
  }
}

// The exact pass over the positions whose key is >= lowkey.  A position is
// kept when its bit in the bitmap was clear, i.e. it is the first position of
// its slot to arrive; kept keys and slots go to the workgroup's dense region
// (D.count holds the lengths) and are counted in the histogram of top digits
// (radix pass 0 of k_mc_tail).  Within a region the order of the kept entries
// depends on the timing of the waves; nothing downstream depends on it (the
// histograms count, the gather ranks ties by key).
__global__ void __launch_bounds__(256) k_mc_dedup(const unsigned* cand, const unsigned long long* pkey, SelBufs D,
                                                  McState* st, unsigned* hist, unsigned* bitmap) {
  constexpr int U = 8;  // position keys a thread reads at once
  __shared__ unsigned h[kRadixBins];
  __shared__ unsigned s_run;
  if (st->skip) return;
  const int tid = threadIdx.x;
  const unsigned long long lowkey = st->lowkey;
  for (int i = tid; i < kRadixBins; i += blockDim.x) h[i] = 0u;
  if (tid == 0) s_run = 0u;
  __syncthreads();
  const unsigned long long n = st->n_pages * kPage;
  const unsigned long long base = blockIdx.x * sel_region(n);
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  // the workgroup visits the positions of a grid-stride loop (the dense
  // region's size assumes it), U strides at a time; the few kept entries
  // take places in the region through a shared counter
  for (unsigned long long i0 = (unsigned long long)blockIdx.x * blockDim.x + tid; i0 < n; i0 += stride * U) {
    unsigned long long key[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned long long i = i0 + (unsigned long long)u * stride;
      key[u] = i < n ? pkey[i] : kKeyExcluded;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (key[u] == kKeyExcluded || key[u] < lowkey) continue;
      const unsigned sl = cand[i0 + (unsigned long long)u * stride];
      const unsigned bit = 1u << (sl & 31);
      if (atomicOr(&bitmap[sl >> 5], bit) & bit) continue;  // an earlier position holds the slot
      atomicAdd(&h[key[u] >> radix_shift(0)], 1u);
      const unsigned at = atomicAdd(&s_run, 1u);
      D.key[base + at] = key[u];
      D.slot[base + at] = sl;
    }
  }
  __syncthreads();
  for (int i = tid; i < kRadixBins; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
  if (tid == 0) D.count[blockIdx.x] = s_run;
}

// The rest of the selection in one workgroup (kTailThreads threads; thread t
// reads the dense region of dedup workgroup t): the radix passes over the
// kept keys, pass 0 from the histogram the exact pass filled (which it
// clears); the chosen set (keys above the threshold, or every kept key when
// there are at most k); the keys equal to the threshold ranked by
// determinant key when only some of them are taken; the chosen set's keys;
// and the bitmap words of the kept slots cleared for the next selection
// (every set bit belongs to a kept slot).  With full = 0 it only chooses the
// digit of pass 0 and leaves the state of the radix select in McState for
// the grid passes 1..5 (k_mc_radix) and the grid gather (k_mc_gather_ties),
// which serve large k: one workgroup's histogram atomics then crowd into a
// few bins.
constexpr int kTailThreads = 1024;
static_assert(kTailThreads == kSelBlocks, "one dense region per tail thread");

// Block-wide: the digit whose bin (of nb, in LDS) holds the need-th largest
// key, the keys in the bins above it, and its count; every thread gets them.
__device__ void tail_find(const unsigned* h, int nb, long long need, int* d_out,
                          unsigned long long* above_out, unsigned* hd_out) {
  __shared__ unsigned long long s_wt[kTailThreads / 64];
  __shared__ unsigned long long s_above;
  __shared__ unsigned s_hd;
  __shared__ int s_d;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  const int per = (nb + blockDim.x - 1) / blockDim.x;  // 2 (11-bit digits) or 1 (the last, 9-bit digit)
  unsigned hv[2] = {0u, 0u};
  unsigned long long run = 0;
  for (int u = 0; u < per; ++u) {
    const int b = tid * per + u;
    hv[u] = b < nb ? h[b] : 0u;
    run += hv[u];
  }
  unsigned long long x = run;  // inclusive suffix over the wave's lanes
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_down(x, o);
    if (lane + o < 64) x += y;
  }
  if (lane == 0) s_wt[w] = x;
  if (tid == 0) s_d = -1;
  __syncthreads();
  unsigned long long acc = x - run;
  for (int q = w + 1; q < nw; ++q) acc += s_wt[q];
  for (int u = per - 1; u >= 0; --u) {
    if ((long long)acc < need && (long long)(acc + hv[u]) >= need) {
      s_d = tid * per + u;
      s_above = acc;
      s_hd = hv[u];
    }
    acc += hv[u];
  }
  __syncthreads();
  *d_out = s_d;
  *above_out = s_above;
  *hd_out = s_hd;
  __syncthreads();
}

// Entries of the thread's dense region, eight loads in flight.
template <class F>
__device__ __forceinline__ void tail_sweep(const SelBufs& D, unsigned long long base, unsigned cnt, F&& f) {
  for (unsigned j0 = 0; j0 < cnt; j0 += 8) {
    unsigned long long kk[8];
    unsigned ss[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      kk[u] = j0 + u < cnt ? D.key[base + j0 + u] : 0ull;
      ss[u] = j0 + u < cnt ? D.slot[base + j0 + u] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j0 + u < cnt) f(kk[u], ss[u]);
  }
}

constexpr int kTailList = 2048;  // bucket entries the tail keeps in LDS
constexpr int kTailMaxK = 256;   // larger k: pass 0 in the tail, passes 1..5 and the gather on the grid

__global__ void __launch_bounds__(kTailThreads) k_mc_tail(const Slot* T, SelBufs D, McState* st, Ctl* ctl,
                                                          unsigned* hist, int64_t* sel_slot, uint64_t* sel_a,
                                                          uint64_t* sel_b, int k, unsigned* bitmap, int full) {
  __shared__ unsigned h[kRadixBins];
  __shared__ unsigned s_ties[kMaxTies];
  __shared__ unsigned long long s_lk[kTailList];
  __shared__ unsigned s_ls[kTailList];
  __shared__ int64_t s_sel[1024];  // k <= 1024
  __shared__ unsigned long long s_red[kTailThreads / 64];
  __shared__ unsigned s_nsel, s_ntie, s_nl;
  if (st->skip) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  const unsigned long long n = st->n_pages * kPage;
  const unsigned long long stride = (unsigned long long)kSelBlocks * 256;  // the dedup launches' grid
  const unsigned long long base = (unsigned long long)tid * ((n + stride - 1) / stride * 256);
  const unsigned cnt = D.count[tid];
  // kept entries in all
  unsigned long long tsum = cnt;
  for (int o = 32; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o);
  if (lane == 0) s_red[w] = tsum;
  for (int i = tid; i < kRadixBins; i += blockDim.x) {
    h[i] = hist[i];
    hist[i] = 0u;
  }
  if (tid == 0) {
    s_nsel = 0u;
    s_ntie = 0u;
    s_nl = 0u;
  }
  __syncthreads();
  unsigned long long total = 0;
  for (int q = 0; q < nw; ++q) total += s_red[q];
  if (total < (unsigned long long)k && st->lowkey > 0ull) {
    // the bound held fewer than k distinct slots, which the repeat count
    // rules out: stop the run rather than choose from an incomplete set
    for (unsigned j = 0; j < cnt; ++j)
      if (bitmap) bitmap[D.slot[base + j] >> 5] = 0u;
    if (tid == 0) {
      ctl->error |= kErrSelect;
      st->skip = 1;  // the rest of this step does nothing
      st->acc_fallback += 1;
    }
    return;
  }
  const bool all = total <= (unsigned long long)k;
  bool done = all, cleared = false, inl = false;
  unsigned long long P = 0, M = 0;
  long long need = k;
  unsigned hd = 0;
  if (!full) {  // pass 0 only; the grid passes go on from McState
    unsigned long long above = 0;
    if (!all) {
      int d;
      tail_find(h, kRadixBins, need, &d, &above, &hd);
      P = (unsigned long long)d << radix_shift(0);
      M = radix_digit_mask(0) << radix_shift(0);
      need -= (long long)above;
      done = (long long)hd == need;
    }
    if (tid == 0) {
      st->prefix = P;
      st->pmask = M;
      st->n_above = above;
      st->need = need;
      st->all = all ? 1 : 0;
      st->done = done ? 1 : 0;
      st->n_total = total;
      st->n_sel = 0;
      st->n_tie = 0;
      st->arrive = 0;
      st->acc_sel += 1;
      st->acc_kept += total;
    }
    return;
  }
  auto clear_word = [&](unsigned sl) {
    if (bitmap) bitmap[sl >> 5] = 0u;  // every set bit belongs to a kept slot
  };
  // radix select of the k-th largest kept key; once the bucket holding it
  // fits in LDS, the keys above it join the chosen set and the bucket moves
  // to LDS, where the remaining passes and the gather run
  for (int pass = 0; pass < kRadixPasses && !done; ++pass) {
    const int sh = radix_shift(pass);
    const unsigned long long dm = radix_digit_mask(pass);
    if (pass > 0) {
      if (!inl && hd <= (unsigned)kTailList) {
        tail_sweep(D, base, cnt, [&](unsigned long long key, unsigned sl) {
          if (!cleared) clear_word(sl);
          const unsigned long long km = key & M;
          if (km > P) {
            const unsigned q = atomicAdd(&s_nsel, 1u);
            if (q < (unsigned)k) s_sel[q] = sl;
          } else if (km == P) {
            const unsigned t = atomicAdd(&s_nl, 1u);
            if (t < (unsigned)kTailList) {
              s_lk[t] = key;
              s_ls[t] = sl;
            }
          }
        });
        cleared = true;
        inl = true;
      }
      __syncthreads();
      for (int i = tid; i < kRadixBins; i += blockDim.x) h[i] = 0u;
      __syncthreads();
      if (inl) {
        for (unsigned t = tid; t < s_nl; t += blockDim.x)
          if ((s_lk[t] & M) == P) atomicAdd(&h[(s_lk[t] >> sh) & dm], 1u);
      } else {
        tail_sweep(D, base, cnt, [&](unsigned long long key, unsigned sl) {
          if (!cleared) clear_word(sl);
          if ((key & M) == P) atomicAdd(&h[(key >> sh) & dm], 1u);
        });
        cleared = true;
      }
      __syncthreads();
    }
    int d;
    unsigned long long above;
    tail_find(h, (int)dm + 1, need, &d, &above, &hd);
    P |= (unsigned long long)d << sh;
    M |= dm << sh;
    need -= (long long)above;
    done = (long long)hd == need;
  }
  // the rest of the chosen set: keys above the threshold, and the bucket
  // when all of it is taken; otherwise the keys equal to the threshold are
  // ties (every key then has all 64 bits fixed)
  auto gather = [&](unsigned long long key, unsigned sl) {
    const unsigned long long km = key & M;
    if (all || km > P || (done && km == P)) {
      const unsigned q = atomicAdd(&s_nsel, 1u);
      if (q < (unsigned)k) s_sel[q] = sl;
    } else if (km == P) {
      const unsigned t = atomicAdd(&s_ntie, 1u);
      if (t < (unsigned)kMaxTies) s_ties[t] = sl;
    }
  };
  if (inl) {
    for (unsigned t = tid; t < s_nl; t += blockDim.x) gather(s_lk[t], s_ls[t]);
  } else {
    tail_sweep(D, base, cnt, [&](unsigned long long key, unsigned sl) {
      if (!cleared) clear_word(sl);
      gather(key, sl);
    });
  }
  __syncthreads();
  unsigned nsel = min(s_nsel, (unsigned)k);
  if (!done) {  // take need of the ties, smallest determinant keys first
    const int nt = (int)min(s_ntie, (unsigned)kMaxTies);
    for (int i = tid; i < nt; i += blockDim.x) {
      const Slot si = T[s_ties[i]];
      int rank = 0;
      for (int j = 0; j < nt; ++j) {
        const Slot sj = T[s_ties[j]];
        if (key_less(sj.ka, sj.kb, si.ka, si.kb)) ++rank;
      }
      if (rank < need && nsel + rank < (unsigned)k) s_sel[nsel + rank] = s_ties[i];
    }
    nsel += (unsigned)min((long long)nt, need);
    __syncthreads();
  }
  const int m = (int)min(nsel, (unsigned)k);
  for (int i = tid; i < m; i += blockDim.x) {
    const int64_t sl = s_sel[i];
    sel_slot[i] = sl;
    const Slot v = T[sl];
    sel_a[i] = v.ka;
    sel_b[i] = v.kb;
  }
  if (tid == 0) {
    st->n_sel = (unsigned long long)m;
    st->acc_sel += 1;
    st->acc_kept += total;
  }
}

// Gather: chosen candidates -> sel_slot, keys equal to the threshold ->
// ties; the last workgroup resolves the ties by key order and fills the keys
// of the chosen set.  Slots shared between workgroups go through
// agent-scope atomics (the XCDs' L2 caches are not coherent).
__global__ void __launch_bounds__(256) k_mc_gather_ties(const Slot* T, SelBufs D, McState* st,
                                                        int64_t* sel_slot, unsigned* ties, uint64_t* sel_a,
                                                        uint64_t* sel_b, int k, unsigned* bitmap) {
  if (st->skip) return;
  const int tid = threadIdx.x;
  const unsigned long long n = st->n_pages * kPage;
  const unsigned long long base = blockIdx.x * sel_region(n);
  const unsigned long long P = st->prefix, M = st->pmask;
  const int all = st->all, done = st->done;
  const unsigned nb = D.count[blockIdx.x];
  for (unsigned j = tid; j < nb; j += blockDim.x) {
    const unsigned long long km = D.key[base + j] & M;
    const unsigned sl = D.slot[base + j];
    if (bitmap) bitmap[sl >> 5] = 0u;  // every set bit belongs to a kept slot
    const bool take = all || km > P || (done && km == P);
    if (take) {
      const unsigned long long q = atomicAdd(&st->n_sel, 1ull);
      if (q < (unsigned long long)k)
        __hip_atomic_store(&sel_slot[q], (int64_t)sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (km == P) {
      const unsigned long long t = atomicAdd(&st->n_tie, 1ull);
      if (t < kMaxTies) __hip_atomic_store(&ties[t], sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (!last_workgroup(&st->arrive)) return;
  __shared__ unsigned long long s_base, s_nsel;
  if (tid == 0) s_nsel = __hip_atomic_load(&st->n_sel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!(all || done)) {
    const long long need = st->need;
    const unsigned long long ntie = __hip_atomic_load(&st->n_tie, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int nt = (int)min(ntie, (unsigned long long)kMaxTies);
    if (tid == 0) s_base = s_nsel;
    __syncthreads();
    for (int i = tid; i < nt; i += blockDim.x) {
      const unsigned ti = __hip_atomic_load(&ties[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const Slot si = T[ti];
      int rank = 0;
      for (int j = 0; j < nt; ++j) {
        const Slot sj = T[__hip_atomic_load(&ties[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)];
        if (key_less(sj.ka, sj.kb, si.ka, si.kb)) ++rank;
      }
      if (rank < need && s_base + rank < (unsigned long long)k)
        __hip_atomic_store(&sel_slot[s_base + rank], (int64_t)ti, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (tid == 0) {
      s_nsel = s_base + (unsigned long long)min((long long)nt, need);
      st->n_sel = s_nsel;
    }
  }
  __syncthreads();
  const int m = (int)min(s_nsel, (unsigned long long)k);
  for (int i = tid; i < m; i += blockDim.x) {
    const int64_t sl = __hip_atomic_load(&sel_slot[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const Slot v = T[sl];
    sel_a[i] = v.ka;
    sel_b[i] = v.kb;
  }
  if (tid == 0) st->arrive = 0;
}

// H_II: block y builds column y (ket = chosen determinant y)
__global__ void __launch_bounds__(256) k_mc_hii(Ham H, const uint64_t* sel_a, const uint64_t* sel_b,
                                                const McState* st, double* hii, int k, unsigned* cnt,
                                                int64_t n_col) {
  __shared__ Lists L;
  __shared__ double s_red[4];
  if (st->skip) return;
  const int m = (int)min(st->n_sel, (unsigned long long)k);
  // the scatter pages' lengths (the selection has read the previous ones):
  // every entry of a chosen column has a position, columns past m none
  const int chunks = (int)((n_col + kPage - 1) / kPage);
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < (int64_t)k * chunks;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = p % chunks;
    cnt[p] = p / chunks < m ? (unsigned)min((int64_t)kPage, n_col - x * kPage) : 0u;
  }
  const int y = blockIdx.x;
  if (y >= m) return;
  const uint64_t a = sel_a[y], b = sel_b[y];
  make_lists_block(a, b, H.N, L);
  __syncthreads();
  double part = 0.0;
  const int nt = diag_terms(L);
  for (int t = threadIdx.x; t < nt; t += blockDim.x) part += diag_term(H, L, t);
  const double diag = wg_sum(part, s_red);
  for (int i = threadIdx.x; i < m; i += blockDim.x)
    hii[(size_t)i * m + y] = sc_entry(H, sel_a[i], sel_b[i], a, b, L, diag);
}

// ---------------------------------------------------------------- scatter, probe half

// Per quarter of a scatter page (a page is one chosen column x one chunk of
// 256 entries): the partial recalculation sum of b_i over the entries outside
// the chosen set, and the probe / atomic / insert counts of both halves.
struct PageStat {
  double recalc;
  unsigned probes, atomics, inserts;
  int err;
};

// What the probe half learnt about one column entry j of chosen column i,
// for the apply half (same page and lane).
struct ScatRec {
  unsigned slot;  // table slot (kinds kRecZero, kRecLive)
  unsigned kind;
  double h;       // H_ji
};
constexpr unsigned kRecNone = 0;  // H_ji = 0, j in the chosen set, or past the column
constexpr unsigned kRecZero = 1;  // stored with c_j = 0
constexpr unsigned kRecLive = 2;  // stored with c_j != 0
constexpr unsigned kRecMiss = 3;  // not stored

// The probe half runs in the workgroups 1.. of an eigen launch while
// workgroup 0 solves the reduced problem: enumerating the chosen columns,
// their Slater-Condon entries and the table lookups need the chosen set but
// not eta.  Only c of the chosen determinants changes during that launch, and
// the probe half neither reads nor marks those (their b is recalculated and
// they join the candidates in the finish), so it sees the table as the
// selection left it.
struct ProbeArgs {
  Ham H;
  uint64_t mask;
  const uint64_t* sel_a;
  const uint64_t* sel_b;
  unsigned* cand;
  PageStat* pstat;
  ScatRec* rec;
  int64_t n_col;
};

// Lookup for the scatter: the key pair in one 16-byte cached load, c only on
// a match.  Within the scatter launch c never changes and keys only appear
// (with c = 0), so a stale "empty" costs nothing: a large update then goes
// through the claiming insert, which sees the current slot, and a small one
// leaves b alone exactly as for an absent key.  A key seen while its beta word
// is still being published is looked up again with coherent loads.
__device__ __forceinline__ int64_t scatter_find(const Slot* __restrict__ T, uint64_t mask, uint64_t a,
                                                uint64_t b, double* c, int* nprobe) {
  uint64_t idx = hash_key(a, b) & mask;
  for (int n = 0; n < kMaxProbe; ++n) {
    const ulonglong2 kk = *reinterpret_cast<const ulonglong2*>(&T[idx]);
    *nprobe = n + 1;
    if (kk.x == kEmpty) return -1;
    if (kk.x == a) {
      if (kk.y == b) {
        *c = T[idx].c;
        return (int64_t)idx;
      }
      if (kk.y == kPending) {
        int probes = 0;
        SlotVal sv;
        const int64_t s = table_find(T, mask, a, b, &probes, &sv);
        if (s >= 0) *c = sv.c;
        *nprobe = n + 1 + probes;
        return s;
      }
    }
    idx = (idx + 1) & mask;
  }
  return -1;
}

// The lists of one chosen determinant built by a group of 256 threads (t is
// the thread's index in the group; threads 0..N-1 must take part, a barrier
// must follow).
__device__ inline void make_lists_group(uint64_t a, uint64_t b, int N, Lists& L, int t) {
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

// ---------------------------------------------------------------- reduced problem

struct EigArgs {
  const Slot* T;
  Slot* Tw;
  const int64_t* sel_slot;
  const double* hii;  // m x m, symmetric
  McState* st;
  Ctl* ctl;
  double* eta_out;
  double* chat_out;  // c_hat of the chosen determinants after the step
  int k;
  double theta, dx_tol;
  double* tr_E;  // optional per-step energy trace
  ProbeArgs P;   // the probe half, run by the other workgroups
  // optional (wall clock): [0] first start, [1] last end of the probe half,
  // [2] start, [3] end of the reduced problem's workgroup
  unsigned long long* ptime;
};

// The reduced matrix A (order n = m + off, off = 1 when the c~ column exists):
//   A_00 = a00, A_0i = A_i0 = a0_i, A_ij = (H_II)_ij.
// y = A x.  H_II (exactly symmetric) is read column-wise so a wave's loads are
// contiguous.  The waves split the work into 64-row blocks times column
// slices; each lane issues eight loads at a time into four independent partial
// sums, and the slices are combined in shared memory (s_part, 16 * 1025
// doubles would not fit, so slices are combined one row block at a time).
__device__ void mc_matvec(const double* __restrict__ hii, int m, int off, double a00,
                          const double* s_a0, const double* s_x, double* s_y, double* s_part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nrb = (m + 63) >> 6;                     // row blocks of H_II
  const int ns = nrb >= nw ? 1 : nw / nrb;           // column slices per row block
  const int span = (m + ns - 1) / ns;
  for (int rb0 = 0; rb0 < nrb; rb0 += nw / ns) {
    // wave wv works on row block rb0 + wv / ns, slice wv % ns
    const int rb = rb0 + wv / ns, sl = wv % ns;
    const int i = rb * 64 + lane;
    double acc = 0.0;
    if (rb < nrb && wv / ns < nw / ns && i < m) {
      const int j0 = sl * span, j1 = min(m, j0 + span);
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int j = j0;
      // eight loads in flight per lane; the four sums take the same terms in
      // the same order as the four-wide loop below
      for (; j + 7 < j1; j += 8) {
        double hv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) hv[u] = hii[(size_t)(j + u) * m + i];
#pragma unroll
        for (int u = 0; u < 8; u += 4) {
          a0 += hv[u] * s_x[off + j + u];
          a1 += hv[u + 1] * s_x[off + j + u + 1];
          a2 += hv[u + 2] * s_x[off + j + u + 2];
          a3 += hv[u + 3] * s_x[off + j + u + 3];
        }
      }
      for (; j + 3 < j1; j += 4) {
        a0 += hii[(size_t)j * m + i] * s_x[off + j];
        a1 += hii[(size_t)(j + 1) * m + i] * s_x[off + j + 1];
        a2 += hii[(size_t)(j + 2) * m + i] * s_x[off + j + 2];
        a3 += hii[(size_t)(j + 3) * m + i] * s_x[off + j + 3];
      }
      for (; j < j1; ++j) a0 += hii[(size_t)j * m + i] * s_x[off + j];
      acc = (a0 + a1) + (a2 + a3);
    }
    if (wv / ns < nw / ns) s_part[(wv % ns) * 64 + (wv / ns) * 64 * ns + lane] = acc;
    __syncthreads();
    // combine: thread t of the first (nw / ns) * 64 threads owns one row
    const int t = threadIdx.x;
    if (t < (nw / ns) * 64) {
      const int rbl = t >> 6, ln = t & 63;
      const int ii = (rb0 + rbl) * 64 + ln;
      if (rb0 + rbl < nrb && ii < m) {
        double sum = 0.0;
        for (int q = 0; q < ns; ++q) sum += s_part[q * 64 + rbl * 64 * ns + ln];
        if (off) sum += s_a0[ii] * s_x[0];
        s_y[off + ii] = sum;
      }
    }
    __syncthreads();
  }
  if (off && threadIdx.x < 64) {
    // row 0: a00 x_0 + a0 . x_I
    double p = 0.0;
    for (int j = lane; j < m; j += 64) p += s_a0[j] * s_x[1 + j];
    for (int o = 32; o > 0; o >>= 1) {
      const double q = __shfl_xor(p, o);
      p = (lane & o) ? (q + p) : (p + q);
    }
    if (lane == 0) s_y[0] = a00 * s_x[0] + p;
  }
}

// Membership of a slot in the chosen set, through an open-addressing set of
// the chosen slots in shared memory (2 kSetSlots >= 2 k entries).
constexpr int kSetSlots = 2048;
__device__ __forceinline__ unsigned set_hash(unsigned long long x) {
  return (unsigned)((x * 0x9e3779b97f4a7c15ull) >> 53);  // 11 bits
}
__device__ inline bool chosen_set_has(const unsigned long long* set, unsigned long long slot) {
  for (unsigned h = set_hash(slot);; h = (h + 1) & (kSetSlots - 1)) {
    const unsigned long long v = set[h];
    if (v == slot) return true;
    if (v == ~0ull) return false;
  }
}

// Orders a wave's shared-memory writes before its later reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups 1.. of an eigen launch, while workgroup 0 solves the reduced
// problem on its own compute unit.  Unless the step is skipped, the probe half
// of the scatter.  Its work is cut into quarter pages (64 entries of one
// chosen column); every wave takes a contiguous range of them and runs with
// no workgroup barrier and no atomic (its determinant lists in its own shared
// memory).  An entry j of column i with H_ji != 0, j outside the chosen set,
// is looked up once; a stored j takes the entry's own position in the page's
// candidate list and adds H_ji c_hat_j to the quarter's recalculation sum;
// its record tells the apply half whether j is stored and whether c_j != 0.
// A determinant reached from several columns appears at several positions:
// the selection's first pass keeps its first occurrence.  No entry is
// inserted during the launch, so a lookup whose first slot holds neither the
// key nor the empty mark is the only one that walks on.
__device__ void mc_probe_phase(const EigArgs& A) {
  __shared__ unsigned long long s_set[kSetSlots];
  __shared__ Lists s_wl[16];
  const ProbeArgs& P = A.P;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t part = blockIdx.x - 1, nparts = gridDim.x - 1;
  if (part == 0 && tid == 0) {  // gather counters of the next selection
    A.st->n_tie = 0;
    A.st->n_dense = 0;
  }
  if (A.st->skip) return;
  if (A.ptime && tid == 0) atomicMin(&A.ptime[0], (unsigned long long)wall_clock64());
  const int chunks = (int)((P.n_col + kPage - 1) / kPage);
  const int m = (int)min(A.st->n_sel, (unsigned long long)A.k);
  for (int i = tid; i < kSetSlots; i += blockDim.x) s_set[i] = ~0ull;
  __syncthreads();
  for (int q = tid; q < m; q += blockDim.x) {
    const unsigned long long v = (unsigned long long)A.sel_slot[q];
    for (unsigned h = set_hash(v);; h = (h + 1) & (kSetSlots - 1))
      if (atomicCAS(&s_set[h], ~0ull, v) == ~0ull) break;
  }
  __syncthreads();
  const long long nw = (long long)nparts * (blockDim.x >> 6);
  const long long wid = (long long)part * (blockDim.x >> 6) + w;
  const long long perc = 4LL * chunks;  // quarter pages per column
  const long long Q = (long long)m * perc;
  const long long q0 = wid * Q / nw, q1 = (wid + 1) * Q / nw;
  Lists& L = s_wl[w];
  int ycur = -1;
  uint64_t a = 0, b = 0;
  for (long long q = q0; q < q1; ++q) {
    const int y = (int)(q / perc);
    const int rem = (int)(q - (long long)y * perc);
    const int x = rem >> 2, qq = rem & 3;
    if (y != ycur) {
      ycur = y;
      a = P.sel_a[y];
      b = P.sel_b[y];
      wave_sync();  // the previous column's lists are no longer read
      make_lists_group(a, b, P.H.N, L, lane);
      wave_sync();
    }
    const size_t pos = (size_t)(y * chunks + x) * kPage + qq * 64 + lane;
    const int64_t e = (int64_t)x * kPage + qq * 64 + lane;
    double recalc = 0.0;
    unsigned probes = 0u;
    if (e < P.n_col) {
      ScatRec rc{0u, kRecNone, 0.0};
      unsigned cslot = kNoCand;
      if (e != 0) {  // entry 0 is the chosen determinant itself
        uint64_t ja = a, jb = b;
        const double Hj = column_entry(P.H, L, a, b, e, 0.0, &ja, &jb);
        if (Hj != 0.0) {
          const uint64_t idx = hash_key(ja, jb) & P.mask;
          const ulonglong2 kk = *reinterpret_cast<const ulonglong2*>(&A.T[idx]);
          int64_t slot = -1;
          probes = 1u;
          if (kk.x == ja && kk.y == jb) {
            slot = (int64_t)idx;
          } else if (kk.x != kEmpty) {
            double cdummy = 0.0;
            int nf = 0;
            slot = scatter_find(A.T, P.mask, ja, jb, &cdummy, &nf);
            probes = (unsigned)nf;
          }
          if (slot < 0) {
            rc = ScatRec{0u, kRecMiss, Hj};
          } else if (!chosen_set_has(s_set, (unsigned long long)slot)) {
            const double cj = A.T[slot].c;
            rc = ScatRec{(unsigned)slot, cj != 0.0 ? kRecLive : kRecZero, Hj};
            recalc = Hj * cj;
            cslot = (unsigned)slot;
          }
        }
      }
      P.rec[pos] = rc;
      P.cand[pos] = cslot;
    }
    for (int offs = 32; offs > 0; offs >>= 1) {
      recalc += __shfl_xor(recalc, offs);
      probes += __shfl_xor(probes, offs);
    }
    if (lane == 0) P.pstat[(size_t)(y * chunks + x) * 4 + qq] = PageStat{recalc, probes, 0u, 0u, 0};
  }
  if (A.ptime) {
    __syncthreads();
    if (tid == 0) atomicMax(&A.ptime[1], (unsigned long long)wall_clock64());
  }
}

// per-step probe-half timestamps: first start (min) and last end (max)
__global__ void k_ptime_init(unsigned long long* ptime, int64_t nsteps) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsteps; i += (int64_t)gridDim.x * blockDim.x) {
    ptime[4 * i] = ~0ull;
    ptime[4 * i + 1] = 0ull;
    ptime[4 * i + 2] = 0ull;
    ptime[4 * i + 3] = 0ull;
  }
}

// The end of the step, shared by both eigen kernels: the new scalars from
// eta (thread i < m holds eta_i, c_i, b_i and (H_II eta)_i), c_hat_I += eta/s',
// the damped step length and the stopping test.
__device__ void mc_step_finish(const EigArgs& A, int m, double s, dd mu, dd al, double gamma,
                               double eta_i, double ci, double bi, double heta_i, int iters,
                               double* s_red) {
  Ctl* ctl = A.ctl;
  const int tid = threadIdx.x;
  const dd ec = wg_sum_dd(two_prod(eta_i, ci), s_red);
  const dd eb = wg_sum_dd(two_prod(eta_i, bi), s_red);
  const dd ee = wg_sum_dd(two_prod(eta_i, eta_i), s_red);
  const dd ehe = wg_sum_dd(two_prod(eta_i, heta_i), s_red);
  // mu' = gamma^2 mu + 2 gamma eta.c_I + eta.eta ;
  // alpha' = gamma^2 alpha + 2 gamma eta.b_I + eta.H_II.eta   (Alg. 2)
  const dd g2 = two_prod(gamma, gamma);
  const dd mu_n = dd_add(dd_add(dd_mul(g2, mu), dd_mul_d(ec, 2.0 * gamma)), ee);
  const dd al_n = dd_add(dd_add(dd_mul(g2, al), dd_mul_d(eb, 2.0 * gamma)), ehe);
  const double s_new = gamma * s;
  if (tid < m) {
    A.eta_out[tid] = eta_i;
    Slot* sl = A.Tw + A.sel_slot[tid];
    const double cn = sl->c + eta_i / s_new;  // c_hat_I += eta / s'
    sl->c = cn;
    A.chat_out[tid] = cn;
  }
  if (tid == 0) {
    ctl->mu_hi = mu_n.hi;
    ctl->mu_lo = mu_n.lo;
    ctl->al_hi = al_n.hi;
    ctl->al_lo = al_n.lo;
    const double E = dd_val(al_n) / dd_val(mu_n);
    ctl->energy = E;
    const double step_norm = sqrt(fmax(0.0, dd_val(ee)));
    ctl->d = (ctl->steps == 0) ? step_norm : A.theta * ctl->d + (1.0 - A.theta) * step_norm;
    if (A.tr_E) A.tr_E[ctl->steps] = E;
    ctl->steps += 1;
    ctl->steps_this_call += 1;
    if (ctl->d < A.dx_tol) ctl->stopped = 1;
    A.st->scale = s_new;
    A.st->inv_scale = 1.0 / s_new;
    A.st->gamma = gamma;
    A.st->eig_iters = iters;
    // doubles reach 2^1023: fold the scale into the table long before that
    A.st->rescale = fabs(log2(fabs(s_new))) > 400.0 ? 1 : 0;
    if (!(fabs(s_new) > 1e-250) || !(E == E)) ctl->error |= kErrNumeric;
  }
}

// Several workgroup sums at once (one barrier pair for all of them), each in
// a fixed order; v[0..NS) per thread in, the totals in every thread out.
template <int NS>
__device__ __forceinline__ void wg_sums(double* v, double* s_red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NS; ++q)
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v[q], off);
      v[q] = (lane & off) ? (o + v[q]) : (v[q] + o);
    }
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NS; ++q) s_red[q * 16 + w] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += s_red[q * 16 + i];
    v[q] = t;
  }
  __syncthreads();
}

// Lowest eigenpair of a symmetric 3 x 3 matrix g (row-major) by cyclic Jacobi
// rotations, one thread; columns whose `use` flag is off are left out (their
// rows and columns are zero and never chosen).  y gets the unit eigenvector.
__device__ inline double sym3_lowest(const double* g_in, const int* use, double* y) {
  double a[3][3], v[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      a[i][j] = (use[i] && use[j]) ? g_in[i * 3 + j] : 0.0;
      v[i][j] = i == j ? 1.0 : 0.0;
    }
  const double scale = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]) + 1e-300;
  for (int sweep = 0; sweep < 12; ++sweep) {
    // quadratic convergence: off-diagonals below 1e-20 of the diagonal change
    // the eigenvalues by (1e-20)^2 relative
    const double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    if (off <= 1e-20 * scale) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; ++k) {  // columns p, q
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - sn * vkq;
          v[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  int best = -1;
  for (int i = 0; i < 3; ++i)
    if (use[i] && (best < 0 || a[i][i] < a[best][best])) best = i;
  for (int k = 0; k < 3; ++k) y[k] = use[k] ? v[k][best] : 0.0;
  return a[best][best];
}

// The reduced problem by LOBPCG (locally optimal block preconditioned
// conjugate gradient, one vector), one workgroup of NT threads (512 for
// k <= 64, 1024 above): from x = [nu; c_I] / |.| with a fixed pseudo-random
// first search direction,
// each iteration takes the Rayleigh-Ritz minimum of A over span{x, w, p}
// with w = D^-1 (A x - theta x) the residual preconditioned by the diagonal
// D = |diag(A) - theta| (floored at 1e-8 (|theta| + 1)) and p the previous
// step.  D must be positive: LOBPCG needs a positive definite
// preconditioner, and the signed diag(A) - theta is indefinite once theta
// has passed a diagonal entry, where the iteration can stall on that
// coordinate for hundreds of iterations.  p and then w are
// orthonormalised against the others (Gram-Schmidt twice, the products with
// A transformed alike) before the 3 x 3 eigenproblem, so the Ritz pair stays
// accurate to rounding.  Stops at |A x - theta x| <= 1e-9 |theta| or after
// kLobpcgMax iterations: the eigenvalue error is quadratic in the residual
// (about 1e-18 theta^2 / gap), and any eta is a valid step, since the
// updates of mu and alpha are exact for the eta taken.  One matrix-vector
// product per iteration; everything else is a handful of workgroup sums.
constexpr int kLobpcgMax = 300;
constexpr double kLobpcgTol = 1e-9;
// a fixed value in [-1/2, 1/2) per row (splitmix64 of the row index)
__device__ __forceinline__ double lobpcg_kick(int r) {
  uint64_t z = (uint64_t)r * 0x9e3779b97f4a7c15ull + 0x632be59bd9b4e019ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1p-53 - 0.5;
}

template <int KM, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 512 ? 4 : 1)))
k_mc_lobpcg(EigArgs A) {
  __shared__ double s_c[KM], s_b[KM], s_a0[KM], s_d[KM + 1];
  __shared__ double s_x[KM + 1], s_w[KM + 1], s_p[KM + 1], s_ax[KM + 1], s_aw[KM + 1], s_ap[KM + 1];
  __shared__ double s_part[NT];
  __shared__ double s_red[16 * 8];
  __shared__ double s_g[9], s_y[3];
  __shared__ int s_use[3];
  if (blockIdx.x > 0) {
    mc_probe_phase(A);
    return;
  }
  Ctl* ctl = A.ctl;
  if (A.st->skip) return;
  const int tid = threadIdx.x;
  if (A.ptime && tid == 0) A.ptime[2] = wall_clock64();
  const int m = (int)min(A.st->n_sel, (unsigned long long)A.k);
  const double s = A.st->scale;
  const dd mu{ctl->mu_hi, ctl->mu_lo}, al{ctl->al_hi, ctl->al_lo};
  const double* hii = A.hii;
  for (int i = tid; i < m; i += blockDim.x) {
    const Slot sl = A.T[A.sel_slot[i]];
    s_c[i] = s * sl.c;
    s_b[i] = s * sl.b;
  }
  __syncthreads();
  // hc = H_II c_I
  mc_matvec(hii, m, 0, 0.0, s_a0, s_c, s_w, s_part);
  __syncthreads();
  const double hc_i = tid < m ? s_w[tid] : 0.0;
  const double ci = tid < m ? s_c[tid] : 0.0, bi = tid < m ? s_b[tid] : 0.0;
  const dd cc = wg_sum_dd(two_prod(ci, ci), s_red);
  const dd cb = wg_sum_dd(two_prod(ci, bi), s_red);
  const dd chc = wg_sum_dd(two_prod(ci, hc_i), s_red);
  const dd nu2 = dd_add(mu, dd{-cc.hi, -cc.lo});
  const dd num = dd_add(dd_add(al, dd{-2.0 * cb.hi, -2.0 * cb.lo}), chc);
  const double nu2v = dd_val(nu2);
  const int off = nu2v > kNu2Floor * dd_val(mu) ? 1 : 0;
  const double nu = off ? sqrt(nu2v) : 0.0;
  const double a00 = off ? dd_val(num) / nu2v : 0.0;
  if (tid < m) {
    s_a0[tid] = off ? (bi - hc_i) / nu : 0.0;
    s_d[off + tid] = hii[(size_t)tid * m + tid];
  }
  if (tid == 0 && off) s_d[0] = a00;
  const int n = m + off;
  if (n == 0) {  // nothing stored and nothing chosen: no step is possible
    if (tid == 0) ctl->stopped = 1;
    return;
  }
  bool have_kick = false;
  // x = [nu; c_I] normalised, and p = a fixed pseudo-random vector
  // orthonormalised against it.  The current point alone can lie in an
  // invariant subspace of A (with n_alpha = n_beta a chosen set closed under
  // the spin flip keeps A's flip parity), from which the iteration would never
  // reach a lowest eigenvector outside it; p gives every eigenvector weight
  // in the first Rayleigh-Ritz space, which also holds x, so theta never
  // exceeds the current point's Rayleigh quotient.
  {
    double v[1] = {0.0};
    for (int r = tid; r < n; r += blockDim.x) {
      const double t = (off && r == 0) ? nu : s_c[r - off];
      s_x[r] = t;
      v[0] += t * t;
    }
    wg_sums<1>(v, s_red);
    const double nrm = sqrt(v[0]);
    double q[2] = {0.0, 0.0};
    for (int r = tid; r < n; r += blockDim.x) {
      const double xr = nrm > 0.0 ? s_x[r] / nrm : (r == 0 ? 1.0 : 0.0);
      const double kr = lobpcg_kick(r);
      s_x[r] = xr;
      s_p[r] = kr;
      q[0] += xr * kr;
      q[1] += kr * kr;
    }
    wg_sums<2>(q, s_red);
    // p - (x.p) x, normalised (|p'|^2 = |p|^2 - (x.p)^2 as |x| = 1)
    const double pp = q[1] - q[0] * q[0];
    const double ip = pp > 1e-28 ? 1.0 / sqrt(pp) : 0.0;
    for (int r = tid; r < n; r += blockDim.x) s_p[r] = (s_p[r] - q[0] * s_x[r]) * ip;
    have_kick = pp > 1e-28;
  }
  __syncthreads();
  mc_matvec(hii, m, off, a00, s_a0, s_p, s_ap, s_part);
  __syncthreads();
  mc_matvec(hii, m, off, a00, s_a0, s_x, s_ax, s_part);
  __syncthreads();
  double theta;
  {
    double v[1] = {0.0};
    for (int r = tid; r < n; r += blockDim.x) v[0] += s_x[r] * s_ax[r];
    wg_sums<1>(v, s_red);
    theta = v[0];
  }
  bool have_p = have_kick;
  int iters = 0;
  for (int it = 0; it < kLobpcgMax; ++it) {
    // residual, its preconditioned form, and x . p (first Gram-Schmidt pass of p)
    double v[2] = {0.0, 0.0};
    const double dfloor = 1e-8 * (fabs(theta) + 1.0);
    for (int r = tid; r < n; r += blockDim.x) {
      const double res = s_ax[r] - theta * s_x[r];
      v[0] += res * res;
      v[1] += s_x[r] * s_p[r];
      s_w[r] = res / fmax(fabs(s_d[r] - theta), dfloor);
    }
    wg_sums<2>(v, s_red);
    iters = it;
    if (sqrt(v[0]) <= kLobpcgTol * fabs(theta)) break;
    // p orthonormalised against x (two passes; the second pass's coefficient
    // and the norm come from one sum, |p''|^2 = |p'|^2 - q'^2 as |x| = 1), A p along
    if (have_p) {
      double q2[2] = {0.0, 0.0};
      for (int r = tid; r < n; r += blockDim.x) {
        const double pr = s_p[r] - v[1] * s_x[r];
        s_p[r] = pr;
        s_ap[r] -= v[1] * s_ax[r];
        q2[0] += s_x[r] * pr;
        q2[1] += pr * pr;
      }
      wg_sums<2>(q2, s_red);
      const double pp = q2[1] - q2[0] * q2[0];
      have_p = pp > 1e-28;
      const double ip = have_p ? 1.0 / sqrt(pp) : 0.0;
      for (int r = tid; r < n; r += blockDim.x) {
        s_p[r] = (s_p[r] - q2[0] * s_x[r]) * ip;
        s_ap[r] = (s_ap[r] - q2[0] * s_ax[r]) * ip;
      }
      __syncthreads();
    }
    // w orthonormalised against x and p (two passes, the norm with the second)
    double q[2] = {0.0, 0.0};
    for (int r = tid; r < n; r += blockDim.x) {
      q[0] += s_x[r] * s_w[r];
      q[1] += s_p[r] * s_w[r];
    }
    wg_sums<2>(q, s_red);
    double q3[3] = {0.0, 0.0, 0.0};
    for (int r = tid; r < n; r += blockDim.x) {
      const double wr = s_w[r] - q[0] * s_x[r] - (have_p ? q[1] * s_p[r] : 0.0);
      s_w[r] = wr;
      q3[0] += s_x[r] * wr;
      q3[1] += s_p[r] * wr;
      q3[2] += wr * wr;
    }
    wg_sums<3>(q3, s_red);
    if (!have_p) q3[1] = 0.0;
    const double ww = q3[2] - q3[0] * q3[0] - q3[1] * q3[1];
    const bool use_w = ww > 1e-28;
    const double inw = use_w ? 1.0 / sqrt(ww) : 0.0;
    for (int r = tid; r < n; r += blockDim.x)
      s_w[r] = (s_w[r] - q3[0] * s_x[r] - (have_p ? q3[1] * s_p[r] : 0.0)) * inw;
    __syncthreads();
    // A w (A p is carried)
    mc_matvec(hii, m, off, a00, s_a0, s_w, s_aw, s_part);
    __syncthreads();
    // Gram matrix of A on [x, w, p]
    double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = tid; r < n; r += blockDim.x) {
      g[0] += s_x[r] * s_ax[r];
      g[1] += s_x[r] * s_aw[r];
      g[2] += s_x[r] * s_ap[r];
      g[3] += s_w[r] * s_aw[r];
      g[4] += s_w[r] * s_ap[r];
      g[5] += s_p[r] * s_ap[r];
    }
    wg_sums<6>(g, s_red);
    if (tid == 0) {
      const double G[9] = {g[0], g[1], g[2], g[1], g[3], g[4], g[2], g[4], g[5]};
      for (int t = 0; t < 9; ++t) s_g[t] = G[t];
      s_use[0] = 1;
      s_use[1] = use_w ? 1 : 0;
      s_use[2] = have_p ? 1 : 0;
      double y[3];
      sym3_lowest(s_g, s_use, y);
      s_y[0] = y[0];
      s_y[1] = y[1];
      s_y[2] = y[2];
    }
    __syncthreads();
    const double y0 = s_y[0], y1 = s_y[1], y2 = s_y[2];
    // p <- y1 w + y2 p, x <- y0 x + p (and the same for the products with A);
    // one sum gives |p|^2, |x|^2 and x . A x
    double nx[3] = {0.0, 0.0, 0.0};
    for (int r = tid; r < n; r += blockDim.x) {
      const double np = y1 * s_w[r] + y2 * s_p[r];
      const double nap = y1 * s_aw[r] + y2 * s_ap[r];
      const double xr = y0 * s_x[r] + np;
      const double axr = y0 * s_ax[r] + nap;
      s_x[r] = xr;
      s_ax[r] = axr;
      s_p[r] = np;
      s_ap[r] = nap;
      nx[0] += np * np;
      nx[1] += xr * xr;
      nx[2] += xr * axr;
    }
    wg_sums<3>(nx, s_red);
    have_p = nx[0] > 1e-28;
    // p kept of unit length, x renormalised against rounding drift; theta
    // its Rayleigh quotient
    const double ipn = have_p ? 1.0 / sqrt(nx[0]) : 0.0;
    const double ixn = 1.0 / sqrt(nx[1]);
    for (int r = tid; r < n; r += blockDim.x) {
      s_p[r] *= ipn;
      s_ap[r] *= ipn;
      s_x[r] *= ixn;
      s_ax[r] *= ixn;
    }
    theta = nx[2] / nx[1];
    __syncthreads();
    iters = it + 1;
  }
  const double lam = theta;
  // z = sqrt(-lambda) x
  const double zscale = lam < 0.0 ? sqrt(-lam) : 0.0;
  for (int r = tid; r < n; r += blockDim.x) s_w[r] = zscale * s_x[r];
  __syncthreads();
  // sign: z_0 >= 0 with the c~ column, else z . c_I >= 0
  double zc[1] = {0.0};
  if (!off)
    for (int r = tid; r < n; r += blockDim.x) zc[0] += s_w[r] * s_c[r];
  wg_sums<1>(zc, s_red);
  const double sgn = off ? (s_w[0] < 0.0 ? -1.0 : 1.0) : (zc[0] < 0.0 ? -1.0 : 1.0);
  const double gamma = off ? sgn * s_w[0] / nu : 1.0;
  double eta_i = 0.0;
  if (tid < m) eta_i = sgn * s_w[off + tid] - gamma * s_c[tid];
  __syncthreads();
  if (tid < m) s_x[tid] = eta_i;
  __syncthreads();
  mc_matvec(hii, m, 0, 0.0, s_a0, s_x, s_w, s_part);
  __syncthreads();
  const double heta_i = tid < m ? s_w[tid] : 0.0;
  mc_step_finish(A, m, s, mu, al, gamma, eta_i, ci, bi, heta_i, iters, s_red);
  if (A.ptime) {
    __syncthreads();
    if (tid == 0) A.ptime[3] = wall_clock64();
  }
}

constexpr int kEigSmall = 64;  // k up to this: the eigen launch has 512 threads, above 1024
// workgroups of an eigen launch (1 solves, the rest run the probe half):
// two per compute unit for k <= kEigSmall (512 threads, at most 128 VGPRs,
// so the probe half has 16 waves per compute unit), one above (1024 threads)
constexpr int kEigGrid = 256;
constexpr int kEigGridSmall = 512;

// ---------------------------------------------------------------- scatter, apply half

// b_hat += H_{:,I} eta / s' under the compression rule (update b_j iff
// c_j != 0 or |eta_i H_ji| >= tau), from the probe half's records: a stored j
// costs one FP64 atomic on its recorded slot (none when c_j = 0 and the
// increment is small); an absent j with a large increment is inserted (its key
// enumerated again) and takes the entry's position in the page's candidate
// list.  grid =
// (column chunks, k), one record per thread.  Entries of the chosen set are
// skipped: their b is recalculated in the finish.  The page's counts are added
// to the probe half's record of its first quarter.
struct ApplyArgs {
  Ham H;
  Slot* T;
  uint64_t mask;
  const uint64_t* sel_a;
  const uint64_t* sel_b;
  const double* eta;
  const McState* st;
  PageStat* pstat;
  const ScatRec* rec;
  unsigned* cand;
  int64_t n_col;
  double tau;
  int k;
};

__global__ void __launch_bounds__(256) k_mc_apply(ApplyArgs A) {
  __shared__ Lists L;
  __shared__ unsigned s_ins, s_probes, s_atomics;
  __shared__ int s_err, s_need;
  if (A.st->skip) return;
  const int y = blockIdx.y;
  const int m = (int)min(A.st->n_sel, (unsigned long long)A.k);
  if (y >= m) return;
  const unsigned page = (unsigned)(y * gridDim.x + blockIdx.x);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.x == 0) {
    s_ins = s_probes = s_atomics = 0u;
    s_err = 0;
    s_need = 0;
  }
  __syncthreads();
  ScatRec r{0u, kRecNone, 0.0};
  if (e < A.n_col) r = A.rec[(size_t)page * kPage + threadIdx.x];
  const double eta = A.eta[y];
  const double coef = eta * A.st->inv_scale;
  const bool big = fabs(eta * r.h) >= A.tau;
  const bool insert = r.kind == kRecMiss && big;
  if (insert) s_need = 1;
  __syncthreads();
  const uint64_t a = A.sel_a[y], b = A.sel_b[y];
  if (s_need) make_lists_block(a, b, A.H.N, L);
  __syncthreads();
  int my_atomics = 0, my_probes = 0, err = 0;
  if (r.kind == kRecLive || (r.kind == kRecZero && big)) {
    atomic_add_f64(&A.T[r.slot].b, r.h * coef);
    my_atomics = 1;
  } else if (insert) {
    uint64_t ja = a, jb = b;
    (void)column_entry(A.H, L, a, b, e, 0.0, &ja, &jb);
    int ins = 0, probes = 0;
    SlotVal sv;
    const int64_t slot = table_upsert(A.T, A.mask, ja, jb, &ins, &probes, &err, &sv);
    my_probes = probes;
    if (slot >= 0) {
      if (ins) atomicAdd(&s_ins, 1u);
      atomic_add_f64(&A.T[slot].b, r.h * coef);
      my_atomics = 1;
      A.cand[(size_t)page * kPage + threadIdx.x] = (unsigned)slot;
    }
  }
  if (err) atomicOr(&s_err, err);
  if (my_probes) atomicAdd(&s_probes, (unsigned)my_probes);
  if (my_atomics) atomicAdd(&s_atomics, (unsigned)my_atomics);
  __syncthreads();
  if (threadIdx.x == 0) {
    PageStat q = A.pstat[(size_t)page * 4];
    q.probes += s_probes;
    q.atomics += s_atomics;
    q.inserts += s_ins;
    q.err |= s_err;
    A.pstat[(size_t)page * 4] = q;
  }
}

// The chosen columns' sums and the end of the step in one launch of k
// workgroups of 256 threads.  Workgroup i < m sums column i's quarter-page
// partials (the part of the recalculated b_i from entries outside the chosen
// set, and the column's counts) in a fixed order, adds (H_II c_hat_I)_i, the
// part from the chosen set with its new coefficients, and stores the result
// in colstat[i] with agent-scope stores.  The last workgroup to arrive then
// sets b_hat_I from them, puts I on its own candidate pages after the
// scatter pages, adds up the scatter's counts and checks the occupancy.
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_agent(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_agent(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256) k_mc_colfinish(const PageStat* pstat, int chunks, PageStat* colstat,
                                                      const double* hii, const double* chat, Slot* T,
                                                      const int64_t* sel_slot, unsigned* cand, unsigned* cnt,
                                                      McState* st, Ctl* ctl, uint64_t max_entries, unsigned page0,
                                                      int k) {
  __shared__ double s_r[4];
  __shared__ unsigned s_pr[4], s_at[4], s_in[4];
  __shared__ int s_er[4];
  __shared__ unsigned long long s_cnt[3];
  __shared__ int s_err;
  if (st->skip) return;
  const int m = (int)min(st->n_sel, (unsigned long long)k);
  const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (i < m) {
    double r = 0.0, rh = 0.0;
    unsigned pr = 0, at = 0, in = 0;
    int er = 0;
    for (int x = tid; x < 4 * chunks; x += blockDim.x) {
      const PageStat q = pstat[(size_t)i * chunks * 4 + x];
      r += q.recalc;
      pr += q.probes;
      at += q.atomics;
      in += q.inserts;
      er |= q.err;
    }
    for (int q = tid; q < m; q += blockDim.x) rh += hii[(size_t)i * m + q] * chat[q];
    r += rh;
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(r, off);
      r = (lane & off) ? (o + r) : (r + o);
      pr += __shfl_xor(pr, off);
      at += __shfl_xor(at, off);
      in += __shfl_xor(in, off);
      er |= __shfl_xor(er, off);
    }
    if (lane == 0) {
      s_r[w] = r;
      s_pr[w] = pr;
      s_at[w] = at;
      s_in[w] = in;
      s_er[w] = er;
    }
    __syncthreads();
    if (tid == 0) {
      PageStat* o = &colstat[i];
      st_agent(&o->recalc, (s_r[0] + s_r[1]) + (s_r[2] + s_r[3]));
      st_agent(&o->probes, s_pr[0] + s_pr[1] + s_pr[2] + s_pr[3]);
      st_agent(&o->atomics, s_at[0] + s_at[1] + s_at[2] + s_at[3]);
      st_agent(&o->inserts, s_in[0] + s_in[1] + s_in[2] + s_in[3]);
      st_agent(reinterpret_cast<unsigned*>(&o->err), (unsigned)(s_er[0] | s_er[1] | s_er[2] | s_er[3]));
    }
  }
  if (!last_workgroup(&st->arrive_cols)) return;
  if (tid == 0) {
    s_cnt[0] = s_cnt[1] = s_cnt[2] = 0;
    s_err = 0;
  }
  __syncthreads();
  {
    unsigned long long pr = 0, at = 0, in = 0;
    int er = 0;
    for (int p = tid; p < m; p += blockDim.x) {
      const PageStat* q = &colstat[p];
      pr += ld_agent(&q->probes);
      at += ld_agent(&q->atomics);
      in += ld_agent(&q->inserts);
      er |= (int)ld_agent(reinterpret_cast<const unsigned*>(&q->err));
    }
    if (pr) atomicAdd(&s_cnt[0], pr);
    if (at) atomicAdd(&s_cnt[1], at);
    if (in) atomicAdd(&s_cnt[2], in);
    if (er) atomicOr(&s_err, er);
  }
  for (int p = tid; p < m; p += blockDim.x) {
    const int64_t slot = sel_slot[p];
    T[slot].b = ld_agent(&colstat[p].recalc);
    cand[(size_t)page0 * kPage + p] = (unsigned)slot;  // the scatter pages never hold the chosen set
  }
  const unsigned npg = (unsigned)((k + kPage - 1) / kPage);
  for (unsigned p = tid; p < npg; p += blockDim.x)
    cnt[page0 + p] = (unsigned)m > p * kPage ? min((unsigned)kPage, (unsigned)m - p * kPage) : 0u;
  __syncthreads();
  if (tid == 0) {
    st->arrive_cols = 0;
    st->last_sel = (unsigned long long)m;
    st->n_sel = 0;
    st->n_pages = (unsigned long long)page0 + npg;
    ctl->probes += s_cnt[0];
    ctl->atomics += s_cnt[1];
    ctl->inserts += s_cnt[2];
    ctl->occupied += s_cnt[2];
    ctl->error |= s_err;
    if (ctl->occupied > max_entries) ctl->error |= kErrTableFull;
  }
}

// fold the lazy scale into every stored entry (only when it drifted far)
__global__ void __launch_bounds__(256) k_mc_rescale(Slot* T, uint64_t nslots, McState* st, int force) {
  const int go = force || st->rescale;
  if (!go) return;
  const double s = st->scale;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (T[i].ka == kEmpty) continue;
    T[i].c *= s;
    T[i].b *= s;
  }
}

__global__ void k_mc_rescale_done(McState* st, int force) {
  if (force || st->rescale) {
    st->scale = 1.0;
    st->inv_scale = 1.0;
    st->rescale = 0;
  }
}

// Inspection: the candidates of the coming selection, compacted, with the
// selection key |4 b_hat + 4 mu c_hat| exactly as the radix select forms it
// (g_key) and the stored c_hat, b_hat.
__global__ void __launch_bounds__(256) k_mc_export_cands(const Slot* T, const unsigned* cand, const unsigned* cnt,
                                                         const McState* st, const Ctl* ctl, uint64_t* keys,
                                                         double* g, double* cv, double* bv, unsigned long long cap,
                                                         unsigned long long* count, unsigned* bitmap) {
  const unsigned long long n = st->n_pages * kPage;
  const double mu = ctl->mu_hi + ctl->mu_lo;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    if ((i & (kPage - 1)) >= cnt[i / kPage]) continue;
    const unsigned sl = cand[i];
    if (sl == kNoCand) continue;
    const unsigned bit = 1u << (sl & 31);
    if (atomicOr(&bitmap[sl >> 5], bit) & bit) continue;  // seen at an earlier position
    const Slot v = T[sl];
    const unsigned long long q = atomicAdd(count, 1ull);
    if (q < cap) {
      keys[2 * q] = v.ka;
      keys[2 * q + 1] = v.kb;
      g[q] = __longlong_as_double((long long)g_key(v, mu));
      cv[q] = v.c;
      bv[q] = v.b;
    }
  }
}
