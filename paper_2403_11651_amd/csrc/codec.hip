// Entropy coding of the quantised latents with the ARM's probabilities, for
// gfx950.
//
// Section II: the latent grids are sent with a range coder driven by the
// auto-regressive model p_psi, which gives the distribution of a latent from
// its already decoded neighbours; Section III-B: the decoder's ARM therefore
// runs latent after latent.  Here:
//  * the probability of a latent is the Laplace model of the training rate,
//    its mean and scale quantised for coding (scale index j = rint(8 (s_c -
//    ln 0.01)), mean c + f / 16), looked up in frequency tables (16-bit
//    total, every symbol at least 1, |d| > 48 escaped and sent as raw bits)
//    that a kernel builds in float64;
//  * the coder is interleaved rANS (32-bit states in [2^23, 2^31), byte
//    renormalisation): each set of latent grids (level 0; levels 1..L-1) has
//    up to 64 states, one per lane of a wave, and one byte stream;
//  * the decode order is a wavefront: step t of a grid decodes (i, t - a i),
//    with a the smallest slope that puts every causal neighbour in an
//    earlier step (2, 3, 4 for 8, 16, 24 neighbours).  The decoder keeps, per
//    row, the last 16 decoded columns in LDS (enough for every context set),
//    evaluates the ARM of all the latents of a step side by side (one thread
//    per row), then the coder wave decodes their symbols.
// The encoder computes the same per-latent ARM with the same code, so
// encoder and decoder agree bit for bit; the ARM here is evaluated with
// explicit fused multiply-adds in a fixed order (no contraction below).
#include "common.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace cc {

namespace {

__device__ __forceinline__ int ceil_div_pos(int a, int b) { return a <= 0 ? 0 : (a + b - 1) / b; }

// Laplace(mu, b) mass of symbol k of a table row (k < CD_ESC: d = k - 48
// over [d - 1/2, d + 1/2]; CD_ESC: both tails), float64.
__device__ double row_mass(int k, double mu, double b) {
  if (k == CD_ESC) return 0.5 * exp((-CD_A - 0.5 - mu) / b) + 0.5 * exp(-(CD_A + 0.5 - mu) / b);
  const double d = k - CD_A;
  const double lo = d - 0.5 - mu, hi = d + 0.5 - mu;
  if (lo >= 0.0) return 0.5 * (exp(-lo / b) - exp(-hi / b));
  if (hi <= 0.0) return 0.5 * (exp(hi / b) - exp(lo / b));
  return 1.0 - 0.5 * exp(lo / b) - 0.5 * exp(-hi / b);
}

__device__ __forceinline__ uint32_t base_freq(int k, double mu, double b) {
  return 1u + (uint32_t)floor(row_mass(k, mu, b) * (double)(CD_TOTAL - CD_NSYM));
}

// The ARM (Table I "C-C-LinR" hidden layers, "C-2-Lin" output) of 32
// latents on v_mfma_f32_32x32x2f32: latent n = lane % 32, held by both
// half-waves g = lane / 32.  Features sit on the MFMA rows; product step q
// takes, in half g, the feature dfeat(q, g) (the row the accumulator q of
// that half holds), so a layer's accumulators are the next layer's B operand
// as they are.  cx[q] is the context feature dfeat(q, g) of the lane's
// latent; A operands come from the LDS weights as W + I (the identity is the
// residual connection), the bias is the accumulators' starting value.  The
// output layer runs on the VALU: each half sums its features in a fixed
// order, then mu = b + (half 0 + half 1) in both halves.  Encoder and decoder
// call this same code, so their results agree bit for bit.
template <int C>
__device__ __forceinline__ void codec_arm_mfma(const float* __restrict__ wl, int nh, const float (&cx)[C / 2],
                                               float& mu, float& s) {
  constexpr int NQ = C / 2;
  const int lane = threadIdx.x & 63, m = lane & 31, g = lane >> 5;
  float h[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) h[q] = cx[q];
  const float* p = wl;
  for (int layer = 0; layer < nh; ++layer) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = dfeat(r, g);
      acc[r] = row < C ? p[C * C + row] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = dfeat(q, g);
      const float a = m < C ? p[m * C + k] + (m == k ? 1.0f : 0.0f) : 0.0f;
      acc = mfma32x32x2(a, h[q], acc);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) h[q] = acc[q] > 0.0f ? acc[q] : 0.0f;
    p += C * C + C;
  }
  float pm = 0.0f, ps = 0.0f;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = dfeat(q, g);
    pm = __builtin_fmaf(p[k], h[q], pm);
    ps = __builtin_fmaf(p[C + k], h[q], ps);
  }
  const float om = __shfl_xor(pm, 32, 64), os = __shfl_xor(ps, 32, 64);
  mu = p[2 * C] + (g == 0 ? pm + om : om + pm);
  s = p[2 * C + 1] + (g == 0 ? ps + os : os + ps);
}

// Context feature dfeat(q, g) of latent (i, jj) of a grid read through
// get(r, c) (zero outside the grid).
template <int C, typename Get>
__device__ __forceinline__ void codec_context(int i, int jj, int w, bool valid, Get get, float (&cx)[C / 2]) {
  const int g = (threadIdx.x & 63) >> 5;
#pragma unroll
  for (int q = 0; q < C / 2; ++q) {
    const int dy = g ? ctx_dy<C>(dfeat(q, 1)) : ctx_dy<C>(dfeat(q, 0));
    const int dx = g ? ctx_dx<C>(dfeat(q, 1)) : ctx_dx<C>(dfeat(q, 0));
    const int r = i + dy, c = jj + dx;
    cx[q] = (valid && r >= 0 && c >= 0 && c < w) ? get(r, c) : 0.0f;
  }
}

// Table row (j, f) and integer mean part c of one latent, from its ARM
// outputs, in float32.
__device__ __forceinline__ void coding_decision(float mu, float s, int& row, int& c) {
  const float sc = (s == s) ? fminf(fmaxf(s, CD_LOG_BMIN), CD_LOG_BMAX) : CD_LOG_BMAX;
  const int j = (int)__builtin_rintf((sc - CD_LOG_BMIN) * (float)CD_SCALE_PER_LN);
  const float mc = (mu == mu) ? fminf(fmaxf(mu, -CD_MU_LIM), CD_MU_LIM) : 0.0f;
  const float fl = floorf(mc);
  const float fr = mc - fl;
  int f = (int)__builtin_rintf(fr * (float)CD_NMU);
  c = (int)fl;
  if (f == CD_NMU) {
    f = 0;
    c += 1;
  }
  row = j * CD_NMU + f;
}

// Escape payload of d (|d| > 48): symbol 0 is the bit length n of v = |d| -
// 48 less one (5 raw bits); then the n - 1 bits of v below its leading one
// in chunks (the first takes (n - 1) mod 8 bits, or 8, the others 8; most
// significant first); the last is the sign (1 raw bit).  payload_count is
// the number of payload symbols; payload_sym gives symbol idx as a raw value
// and its bit count.
__device__ __forceinline__ int payload_count(int d) {
  const uint32_t v = (uint32_t)(d < 0 ? -d : d) - CD_A;
  const int r = 31 - __builtin_clz(v);  // bits below the leading one
  return 2 + (r + 7) / 8;
}

__device__ __forceinline__ void payload_sym(int d, int idx, uint32_t& val, int& bits) {
  const uint32_t v = (uint32_t)(d < 0 ? -d : d) - CD_A;
  const int r = 31 - __builtin_clz(v);
  const int nch = (r + 7) / 8;
  if (idx == 0) {
    val = (uint32_t)r;
    bits = 5;
  } else if (idx <= nch) {
    const int first = (r & 7) ? (r & 7) : 8;
    const int size = idx == 1 ? first : 8;
    const int shift = r - first - 8 * (idx - 1);
    val = (v >> shift) & ((1u << size) - 1u);
    bits = size;
  } else {
    val = d < 0 ? 1u : 0u;
    bits = 1;
  }
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
  return v;
}

// Lanes below this one (mbcnt) with their bit set in a 64-bit wave mask.
__device__ __forceinline__ int count_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t load_u32_bytes(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

}  // namespace

// ---------------------------------------------------------------- tables

// One thread per table row (j, f): frequencies 1 + floor(P (2^16 - 98)) of
// the Laplace(f / 16, b_j) masses, the remainder added to the first most
// frequent symbol; stored as cumulative frequencies (CD_ROW per row).
// Thread 0 also clears the encoder's flags (meta may be null).
__global__ void codec_table_kernel(uint32_t* cum, uint16_t* cum16, uint32_t* meta) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row == 0 && meta) {
    meta[CD_META_BAD] = 0u;
    meta[CD_META_OVF] = 0u;
  }
  if (row >= CD_NSCALE * CD_NMU) return;
  const int j = row / CD_NMU, f = row % CD_NMU;
  const double b = exp((double)CD_LOG_BMIN + (double)j / CD_SCALE_PER_LN);
  const double mu = (double)f / CD_NMU;
  uint32_t sum = 0, best = 0;
  int arg = 0;
  for (int k = 0; k < CD_NSYM; ++k) {
    const uint32_t fk = base_freq(k, mu, b);
    sum += fk;
    if (fk > best) {
      best = fk;
      arg = k;
    }
  }
  const uint32_t left = CD_TOTAL - sum;
  uint32_t* out = cum + (size_t)row * CD_ROW;
  uint16_t* o16 = cum16 ? cum16 + (size_t)row * CD_ROW16 : nullptr;
  uint32_t run = 0;
  for (int k = 0; k < CD_NSYM; ++k) {
    out[k] = run;
    if (o16) o16[k] = (uint16_t)run;
    run += base_freq(k, mu, b) + (k == arg ? left : 0u);
  }
  out[CD_NSYM] = run;
  if (o16)
    for (int k = CD_NSYM; k < CD_ROW16; ++k) o16[k] = 0xFFFFu;
}

// ---------------------------------------------------------------- encoder

// One wave per 32 consecutive latents of the packed pyramid (latent n of
// the group on lane n and lane n + 32): the ARM of each latent's (known)
// context, the coding decision, and d = y_hat - c.  A latent that is not an
// integer of magnitude <= 2^20 marks meta[CD_META_BAD].
template <int C>
__global__ void __launch_bounds__(256) codec_params_kernel(CodecArgs a) {
  __shared__ float wl[3 * (24 * 24 + 24) + 2 * 24 + 2];
  const int n_arm = a.NH * (C * C + C) + 2 * C + 2;
  for (int k = threadIdx.x; k < n_arm; k += blockDim.x) wl[k] = a.w[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int q = (blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * 32 + (lane & 31);
  const bool valid = q < a.geo.n_lat;
  int lv = 0;
  while (valid && lv + 1 < a.geo.L && q >= a.geo.loff[lv + 1]) ++lv;
  const int w = a.geo.lw[lv], off = a.geo.loff[lv];
  const int i = valid ? (q - off) / w : 0, jj = valid ? (q - off) - i * w : 0;
  const float raw = valid ? a.yq[q] : 0.0f;
  const bool ok = raw == __builtin_rintf(raw) && fabsf(raw) <= (float)CD_YQ_LIM;
  if (valid && !ok) a.meta[CD_META_BAD] = 1u;
  float cx[C / 2];
  codec_context<C>(i, jj, w, valid, [&](int r, int c) {
    const float y = a.yq[off + r * w + c];
    return (float)(int)fminf(fmaxf(y, -(float)CD_YQ_LIM), (float)CD_YQ_LIM);  // canonical integer value
  }, cx);
  float mu, s;
  codec_arm_mfma<C>(wl, a.NH, cx, mu, s);
  int row, c;
  coding_decision(mu, s, row, c);
  if (valid && lane < 32) {
    a.tbl[q] = (uint16_t)row;
    a.dsym[q] = ok ? (int)raw - c : 0;
  }
}

// One wave per set: the rounds of the set in reverse decode order; in each
// round the states that must renormalise emit their bytes (states in
// descending order), then every participating state encodes its symbol.
__global__ void __launch_bounds__(64) codec_encode_kernel(CodecArgs a) {
  const int set = blockIdx.x, lane = threadIdx.x;
  const CodecSet S = a.set[set];
  const int n = S.n_lanes, slope = a.slope;
  uint8_t* __restrict__ em = a.emit[set];
  const int64_t cap = a.emit_cap[set];
  uint32_t x = CD_RANS_L;
  int64_t pos = 0;
  bool ovf = false;
  for (int lv = S.lv1 - 1; lv >= S.lv0; --lv) {
    const int h = a.geo.lh[lv], w = a.geo.lw[lv], off = a.geo.loff[lv];
    for (int t = w - 1 + slope * (h - 1); t >= 0; --t) {
      const int i_lo = ceil_div_pos(t - (w - 1), slope), i_hi = min(h - 1, t / slope);
      if (i_lo > i_hi) continue;
      for (int g = i_hi / n; g >= i_lo / n; --g) {
        const int i = g * n + lane;
        const bool act = lane < n && i >= i_lo && i <= i_hi;
        int row = 0, d = 0, ns = 0;
        if (act) {
          const int q = off + i * w + (t - slope * i);
          row = a.tbl[q];
          d = a.dsym[q];
          ns = (d >= -CD_A && d <= CD_A) ? 1 : 1 + payload_count(d);
        }
        const uint32_t* __restrict__ crow = a.cum + (size_t)row * CD_ROW;
        const int nmax = wave_max_i(ns);
        for (int r = nmax - 1; r >= 0; --r) {
          const bool part = r < ns;
          uint32_t cm = 0, fr = 1;
          if (part) {
            if (r == 0) {
              const int k = (d >= -CD_A && d <= CD_A) ? d + CD_A : CD_ESC;
              cm = crow[k];
              fr = crow[k + 1] - cm;
            } else {
              uint32_t val;
              int bits;
              payload_sym(d, r - 1, val, bits);
              cm = val << (CD_PREC - bits);
              fr = 1u << (CD_PREC - bits);
            }
          }
          bool e0 = false, e1 = false;
          if (part) {
            const uint64_t xm = (uint64_t)fr << (23 - CD_PREC + 8);  // (L >> PREC) << 8, times the frequency
            e0 = (uint64_t)x >= xm;
            e1 = (uint64_t)x >= (xm << 8);
          }
          const int k = (int)e0 + (int)e1;
          // bytes of the lanes above this one (they emit first), and in all
          const uint64_t m0 = __ballot(e0), m1 = __ballot(e1);
          const int total = __popcll(m0) + __popcll(m1);
          const int above = total - count_below(m0) - count_below(m1) - k;
          const int64_t at = pos + above;
          if (k > 0) {
            if (at + k <= cap) {
              em[at] = (uint8_t)(x & 0xFFu);
              if (k == 2) em[at + 1] = (uint8_t)((x >> 8) & 0xFFu);
            } else {
              ovf = true;
            }
            x >>= 8 * k;
          }
          pos += total;
          if (part) x = ((x / fr) << CD_PREC) + (x % fr) + cm;
        }
      }
    }
  }
  if (lane == 0) a.meta[set] = (uint32_t)min<int64_t>(pos, 0xFFFFFFFFll);
  if (lane < n) a.meta[2 + set * CD_LANES + lane] = x;
  if (ovf) a.meta[CD_META_OVF] = 1u;
}

// The bitstream: "CCR1", u32 sets, u32 bytes of each set, u32 final states
// (n_lanes per set), then each set's bytes (the emission reversed).
// out_nbytes: the size; 0 for invalid latents; -size when out is too small
// (nothing written).
__global__ void codec_pack_kernel(CodecArgs a) {
  const int ns = a.n_sets;
  int64_t hdr = 8 + 4 * ns;
  int64_t total = hdr;
  int64_t sbase[CD_MAX_SETS], scount[CD_MAX_SETS];
  int lane_base[CD_MAX_SETS];
  int lanes = 0;
  for (int s = 0; s < ns; ++s) {
    lane_base[s] = lanes;
    lanes += a.set[s].n_lanes;
  }
  total += 4 * lanes;
  for (int s = 0; s < ns; ++s) {
    scount[s] = a.meta[s];
    sbase[s] = total;
    total += scount[s];
  }
  const bool bad = a.meta[CD_META_BAD] != 0u || a.meta[CD_META_OVF] != 0u;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) *a.out_nbytes = bad ? 0 : (total <= a.out_cap ? total : -total);
  if (bad || total > a.out_cap) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t head = hdr + 4 * lanes;
  for (int64_t b = gid; b < total; b += stride) {
    uint8_t v;
    if (b < head) {
      const int word = (int)(b >> 2), sh = 8 * (int)(b & 3);
      uint32_t u;
      if (word == 0) {
        u = CD_MAGIC;
      } else if (word == 1) {
        u = (uint32_t)ns;
      } else if (word < 2 + ns) {
        u = (uint32_t)scount[word - 2];
      } else {
        int st = word - 2 - ns, s = 0;
        while (s + 1 < ns && st >= lane_base[s + 1]) ++s;
        u = a.meta[2 + s * CD_LANES + (st - lane_base[s])];
      }
      v = (uint8_t)(u >> sh);
    } else {
      int s = 0;
      while (s + 1 < ns && b >= sbase[s + 1]) ++s;
      const int64_t k = b - sbase[s];
      v = a.emit[s][scount[s] - 1 - k];
    }
    a.out[b] = v;
  }
}

// ---------------------------------------------------------------- decoder

// One work-group of 512 threads per set, wave 0 holds the set's
// coder states.  A step's latents are taken in chunks of at most CD_SLOTS
// rows (rows ascending, so the decode order is kept): the ARM of every latent
// of the chunk (32 rows per wave on the matrix cores, weights staged in LDS,
// context from the ring of decoded values), its coding decision and a copy
// of its table row (uint16) into an LDS slot; then the coder wave decodes the
// chunk's symbols with a binary search in the slots, reading the byte stream
// through an LDS cache.
// status[set]: 0 on success, 1 header mismatch, 2 stream overrun, 4 the
// stream or the final states disagree with the problem.
constexpr int CD_SCACHE_WORDS = 512;    // stream cache of the coder wave: 2 KB

size_t codec_decode_lds_bytes(int rows_max, int n_arm) {
  return (size_t)rows_max * CD_RING * sizeof(float) + (size_t)CD_SLOTS * (sizeof(int) + CD_ROW16 * 2) +
         (size_t)((n_arm + 3) / 4 * 4) * sizeof(float) + CD_SCACHE_WORDS * sizeof(uint32_t);
}

template <int C>
__global__ void __launch_bounds__(512) codec_decode_kernel(CodecArgs a) {
  extern __shared__ float smem[];
  const int n_arm = a.NH * (C * C + C) + 2 * C + 2;
  float* ring = smem;
  uint16_t* slots = (uint16_t*)(ring + (size_t)a.rows_max * CD_RING);    // [CD_SLOTS][CD_ROW16]
  int* cval = (int*)(slots + (size_t)CD_SLOTS * CD_ROW16);                // [CD_SLOTS]
  float* wl = (float*)(cval + CD_SLOTS);
  uint32_t* scache = (uint32_t*)(wl + (n_arm + 3) / 4 * 4);
  const int set = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nt = blockDim.x;
  const CodecSet S = a.set[set];
  const int n = S.n_lanes, slope = a.slope, ns = a.n_sets;
  const uint8_t* __restrict__ in = a.in;

  for (int k = tid; k < n_arm; k += nt) wl[k] = a.w[k];

  // header (every thread reads the same words)
  int64_t head = 8 + 4 * ns;
  int lane_base = 0, lanes = 0;
  for (int s = 0; s < ns; ++s) {
    if (s == set) lane_base = lanes;
    lanes += a.set[s].n_lanes;
  }
  head += 4 * lanes;
  int status = 0;
  int64_t count = 0, start = head, total = head;
  if (a.in_bytes < head || load_u32_bytes(in) != CD_MAGIC || load_u32_bytes(in + 4) != (uint32_t)ns) {
    status = 1;
  } else {
    for (int s = 0; s < ns; ++s) {
      const int64_t cs = load_u32_bytes(in + 8 + 4 * s);
      if (s < set) start += cs;
      if (s == set) count = cs;
      total += cs;
    }
    if (total != a.in_bytes) status = 1;
  }
  if (status) {
    if (tid == 0) a.status[set] = status;
    return;
  }
  uint32_t x = CD_RANS_L;
  if (wave == 0 && lane < n) x = load_u32_bytes(in + 8 + 4 * ns + 4 * (lane_base + lane));
  int64_t pos = 0;                        // stream bytes consumed (wave 0, uniform)
  int64_t c_lo = 0, c_hi = 0;             // the cache holds in[c_lo, c_hi) (absolute offsets)

  // the stream cache covers at least [pos, pos + 128) of the stream
  auto ensure = [&]() {
    const int64_t need = start + pos;
    if (need >= c_lo && need + 128 <= c_hi) return;
    c_lo = need & ~(int64_t)3;
    c_hi = c_lo + 4 * CD_SCACHE_WORDS;
    uint32_t v[CD_SCACHE_WORDS / 64];
#pragma unroll
    for (int m = 0; m < CD_SCACHE_WORDS / 64; ++m) {
      const int64_t o = c_lo + 4 * (lane + 64 * m);
      v[m] = 0;
      if (o + 4 <= a.in_bytes) {
        v[m] = *(const uint32_t*)(in + o);
      } else {
        for (int b = 0; b < 4; ++b)
          if (o + b < a.in_bytes) v[m] |= (uint32_t)in[o + b] << (8 * b);
      }
    }
#pragma unroll
    for (int m = 0; m < CD_SCACHE_WORDS / 64; ++m) scache[lane + 64 * m] = v[m];
    wave_lds_sync();
  };
  auto cached_byte = [&](int64_t at) -> uint32_t {
    const int64_t o = start + at - c_lo;
    return (scache[o >> 2] >> (8 * (o & 3))) & 0xFFu;
  };
  // renormalisation after a round: states below 2^23 read one or two bytes,
  // state after state in ascending order (wave 0 only)
  auto refill = [&](bool part) {
    const bool r0 = part && x < CD_RANS_L, r1 = part && x < (CD_RANS_L >> 8);
    const int k = (int)r0 + (int)r1;
    const uint64_t m0 = __ballot(r0), m1 = __ballot(r1);
    const int tot = __popcll(m0) + __popcll(m1);
    if (tot > 0) {
      ensure();
      const int64_t at = pos + count_below(m0) + count_below(m1);
      if (k > 0) {
        uint32_t b0 = 0, b1 = 0;
        if (at + k <= count) {
          b0 = cached_byte(at);
          if (k == 2) b1 = cached_byte(at + 1);
        } else {
          status |= 2;
        }
        x = (x << 8) | b0;
        if (k == 2) x = (x << 8) | b1;
      }
      pos += tot;
    }
  };
  // one raw symbol of `bits` bits
  auto raw = [&](bool part, int bits) -> uint32_t {
    uint32_t v = 0;
    if (part) {
      const uint32_t slot = x & (CD_TOTAL - 1u);
      v = slot >> (CD_PREC - bits);
      x = (1u << (CD_PREC - bits)) * (x >> CD_PREC) + (slot & ((1u << (CD_PREC - bits)) - 1u));
    }
    refill(part);
    return v;
  };
  __syncthreads();  // ARM weights staged

  for (int lv = S.lv0; lv < S.lv1; ++lv) {
    const int h = a.geo.lh[lv], w = a.geo.lw[lv], off = a.geo.loff[lv];
    const int T = w + slope * (h - 1);
    for (int t = 0; t < T; ++t) {
      const int i_lo = ceil_div_pos(t - (w - 1), slope), i_hi = min(h - 1, t / slope);
      // chunks of CD_SLOTS rows starting on group boundaries (CD_SLOTS is a
      // multiple of the group size n when n = 64; a set with fewer states
      // has fewer than 64 rows, so one chunk), so every group is one round
      for (int cb = i_lo / n * n; cb <= i_hi; cb += CD_SLOTS) {
        const int c_lo_row = max(i_lo, cb), c_hi_row = min(i_hi, cb + CD_SLOTS - 1);
        // ARM, decision and table row of every latent of the chunk: slices of
        // 32 rows, one per wave
        const int nsl = (c_hi_row - c_lo_row) / 32 + 1;
        for (int sl = wave; sl < nsl; sl += nt / 64) {
          const int i = c_lo_row + 32 * sl + (lane & 31);
          const bool valid = i <= c_hi_row;
          const int jj = t - slope * i;
          float cx[C / 2];
          codec_context<C>(i, jj, w, valid, [&](int r, int c) { return ring[r * CD_RING + (c & (CD_RING - 1))]; },
                           cx);
          float mu, s;
          codec_arm_mfma<C>(wl, a.NH, cx, mu, s);
          int row, c;
          coding_decision(mu, s, row, c);
          if (valid) {
            // the table row into the latent's slot: 13 16-byte pieces, 7 by
            // one half-wave and 6 by the other
            const int g = lane >> 5;
            const uint4* __restrict__ src = (const uint4*)(a.cum16 + (size_t)row * CD_ROW16);
            uint4* dst = (uint4*)(slots + (size_t)(i - cb) * CD_ROW16);
            constexpr int NP = CD_ROW16 / 8, NH0 = (NP + 1) / 2;
            const int base = g * NH0;
            uint4 rv[NH0];
#pragma unroll
            for (int m = 0; m < NH0; ++m) rv[m] = src[min(base + m, NP - 1)];  // the last piece twice in half 1
#pragma unroll
            for (int m = 0; m < NH0; ++m) dst[min(base + m, NP - 1)] = rv[m];
            if (g == 0) cval[i - cb] = c;
          }
        }
        __syncthreads();
        if (wave == 0) {
          for (int g = c_lo_row / n; g <= c_hi_row / n; ++g) {
            const int i = g * n + lane;
            const bool act = lane < n && i >= c_lo_row && i <= c_hi_row;
            int c = 0, k = 0;
            if (act) {
              c = cval[i - cb];
              const uint16_t* cr = slots + (size_t)(i - cb) * CD_ROW16;
              const uint32_t slot = x & (CD_TOTAL - 1u);
              // largest k in [0, 97] with cum[k] <= slot (cum[0] = 0): first
              // among d = -4 .. 4 (entries 44 .. 53, read at once), else by
              // bisection
              constexpr int K0 = CD_A - 4, NWIN = 10;
              uint32_t wv[NWIN];
#pragma unroll
              for (int q = 0; q < NWIN; ++q) wv[q] = cr[K0 + q];
              if (slot >= wv[0] && slot < wv[NWIN - 1]) {
                int m = 0;
#pragma unroll
                for (int q = 1; q < NWIN - 1; ++q) m += slot >= wv[q] ? 1 : 0;
                k = K0 + m;
              } else {
                int lo = slot >= wv[NWIN - 1] ? K0 + NWIN - 1 : 0;
#pragma unroll
                for (int step = 64; step >= 1; step >>= 1)
                  if (lo + step < CD_NSYM && (uint32_t)cr[lo + step] <= slot) lo += step;
                k = lo;
              }
              const uint32_t cm = cr[k];
              const uint32_t cn = k + 1 < CD_NSYM ? (uint32_t)cr[k + 1] : CD_TOTAL;
              x = (cn - cm) * (x >> CD_PREC) + slot - cm;
            }
            refill(act);
            const bool esc = act && k == CD_ESC;
            int d = k - CD_A;
            if (__any(esc)) {
              const int r = (int)raw(esc, 5);           // bits below the leading one
              const int nch = (r + 7) / 8, first = (r & 7) ? (r & 7) : 8;
              uint32_t v = 1u, neg = 0u;
              for (int qq = 0; __any(esc && qq <= nch); ++qq) {
                const bool part = esc && qq <= nch;
                const int bits = qq < nch ? (qq == 0 ? first : 8) : 1;
                const uint32_t got = raw(part, bits);
                if (part) {
                  if (qq == nch) neg = got;
                  else v = (v << bits) | got;
                }
              }
              if (esc) d = neg ? -(int)(v + CD_A) : (int)(v + CD_A);
            }
            if (act) {
              const int jj = t - slope * i;
              const float yv = (float)(c + d);
              ring[i * CD_RING + (jj & (CD_RING - 1))] = yv;
              a.yq_out[off + (size_t)i * w + jj] = yv;
            }
          }
        }
        __syncthreads();
      }
    }
  }
  if (wave == 0) {
    const bool end_ok = pos == count && (lane >= n || x == CD_RANS_L);
    if (!__all(end_ok)) status |= 4;
    status = wave_max_i(status);
    if (lane == 0) a.status[set] = status;
  }
}

const void* codec_params_kernel_for(int C) {
  switch (C) {
    case 8: return (const void*)codec_params_kernel<8>;
    case 16: return (const void*)codec_params_kernel<16>;
    case 24: return (const void*)codec_params_kernel<24>;
  }
  return nullptr;
}

const void* codec_decode_kernel_for(int C) {
  switch (C) {
    case 8: return (const void*)codec_decode_kernel<8>;
    case 16: return (const void*)codec_decode_kernel<16>;
    case 24: return (const void*)codec_decode_kernel<24>;
  }
  return nullptr;
}

}  // namespace cc
