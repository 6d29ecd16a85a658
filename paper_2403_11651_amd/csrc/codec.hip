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

// The ARM of one latent from its context (Table I "C-C-LinR" hidden layers,
// "C-2-Lin" output), float32 with a fixed operation order.
template <int C>
__device__ __forceinline__ void codec_arm(const float* __restrict__ w, int nh, const float (&ctx)[C], float& mu,
                                          float& s) {
  float h[C];
#pragma unroll
  for (int k = 0; k < C; ++k) h[k] = ctx[k];
  const float* p = w;
  for (int layer = 0; layer < nh; ++layer) {
    float o[C];
#pragma unroll
    for (int r = 0; r < C; ++r) {
      float acc = p[C * C + r];
#pragma unroll
      for (int k = 0; k < C; ++k) acc = __builtin_fmaf(p[r * C + k], h[k], acc);
      acc = acc + h[r];
      o[r] = acc > 0.0f ? acc : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < C; ++r) h[r] = o[r];
    p += C * C + C;
  }
  float m = p[2 * C], t = p[2 * C + 1];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    m = __builtin_fmaf(p[k], h[k], m);
    t = __builtin_fmaf(p[C + k], h[k], t);
  }
  mu = m;
  s = t;
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

// inclusive sum over lanes >= lane
__device__ __forceinline__ int suffix_sum(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_down(v, o, 64);
    if (lane + o < 64) v += u;
  }
  return v;
}

// inclusive sum over lanes <= lane
__device__ __forceinline__ int prefix_sum(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
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
__global__ void codec_table_kernel(uint32_t* cum, uint32_t* meta) {
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
  uint32_t run = 0;
  for (int k = 0; k < CD_NSYM; ++k) {
    out[k] = run;
    run += base_freq(k, mu, b) + (k == arg ? left : 0u);
  }
  out[CD_NSYM] = run;
}

// ---------------------------------------------------------------- encoder

// One thread per latent: the ARM of its (known) context, the coding
// decision, and d = y_hat - c.  A latent that is not an integer of
// magnitude <= 2^20 marks meta[CD_META_BAD].
template <int C>
__global__ void __launch_bounds__(256) codec_params_kernel(CodecArgs a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.geo.n_lat) return;
  int lv = 0;
  while (lv + 1 < a.geo.L && q >= a.geo.loff[lv + 1]) ++lv;
  const int w = a.geo.lw[lv], h = a.geo.lh[lv], off = a.geo.loff[lv];
  const int i = (q - off) / w, jj = (q - off) - i * w;
  const float raw = a.yq[q];
  const bool ok = raw == __builtin_rintf(raw) && fabsf(raw) <= (float)CD_YQ_LIM;
  if (!ok) a.meta[CD_META_BAD] = 1u;
  float ctx[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const int r = i + ctx_dy<C>(k), c = jj + ctx_dx<C>(k);
    float v = 0.0f;
    if (r >= 0 && c >= 0 && c < w) {
      const float y = a.yq[off + r * w + c];
      v = (float)(int)fminf(fmaxf(y, -(float)CD_YQ_LIM), (float)CD_YQ_LIM);  // canonical integer value
    }
    ctx[k] = v;
  }
  (void)h;
  float mu, s;
  codec_arm<C>(a.w, a.NH, ctx, mu, s);
  int row, c;
  coding_decision(mu, s, row, c);
  a.tbl[q] = (uint16_t)row;
  a.dsym[q] = ok ? (int)raw - c : 0;
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
          int k = 0;
          if (part) {
            const uint64_t xm = (uint64_t)fr << (23 - CD_PREC + 8);  // (L >> PREC) << 8, times the frequency
            k = ((uint64_t)x >= xm) + ((uint64_t)x >= (xm << 8));
          }
          const int incl = suffix_sum(k, lane);
          const int total = __shfl(incl, 0, 64);
          const int64_t at = pos + (incl - k);
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

// One work-group per set (blockDim a multiple of 64; thread tid evaluates
// the ARM for rows tid, tid + blockDim, ...), wave 0 holds the set's coder
// states.  Dynamic LDS: rows_max x CD_RING decoded values, then rows_max
// (table row, c) pairs handed from the ARM threads to the coder wave.
// status[set]: 0 on success, 1 header mismatch, 2 stream overrun, 4 the
// stream or the final states disagree with the problem.
template <int C>
__global__ void __launch_bounds__(1024) codec_decode_kernel(CodecArgs a) {
  extern __shared__ float smem[];
  float* ring = smem;
  int2* hand = (int2*)(ring + (size_t)a.rows_max * CD_RING);
  const int set = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nt = blockDim.x;
  const CodecSet S = a.set[set];
  const int n = S.n_lanes, slope = a.slope, ns = a.n_sets;
  const uint8_t* __restrict__ in = a.in;

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
  const uint8_t* __restrict__ stream = in + start;
  uint32_t x = CD_RANS_L;
  if (wave == 0 && lane < n) x = load_u32_bytes(in + 8 + 4 * ns + 4 * (lane_base + lane));
  int64_t pos = 0;

  // renormalisation after a round: states below 2^23 read one or two bytes,
  // state after state in ascending order (wave 0 only)
  auto refill = [&](bool part) {
    const int k = part ? (int)(x < CD_RANS_L) + (int)(x < (CD_RANS_L >> 8)) : 0;
    const int incl = prefix_sum(k, lane);
    const int tot = __shfl(incl, 63, 64);
    const int64_t at = pos + (incl - k);
    if (k > 0) {
      uint32_t b0 = 0, b1 = 0;
      if (at + k <= count) {
        b0 = stream[at];
        if (k == 2) b1 = stream[at + 1];
      } else {
        status |= 2;
      }
      x = (x << 8) | b0;
      if (k == 2) x = (x << 8) | b1;
    }
    pos += tot;
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

  for (int lv = S.lv0; lv < S.lv1; ++lv) {
    const int h = a.geo.lh[lv], w = a.geo.lw[lv], off = a.geo.loff[lv];
    const int T = w + slope * (h - 1);
    for (int t = 0; t < T; ++t) {
      const int i_lo = ceil_div_pos(t - (w - 1), slope), i_hi = min(h - 1, t / slope);
      // ARM of every latent of the step (context from the ring of decoded values)
      for (int i = i_lo + ((tid - i_lo) % nt + nt) % nt; i <= i_hi; i += nt) {
        const int jj = t - slope * i;
        float ctx[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
          const int r = i + ctx_dy<C>(k), c = jj + ctx_dx<C>(k);
          ctx[k] = (r >= 0 && c >= 0 && c < w) ? ring[r * CD_RING + (c & (CD_RING - 1))] : 0.0f;
        }
        float mu, s;
        codec_arm<C>(a.w, a.NH, ctx, mu, s);
        int row, c;
        coding_decision(mu, s, row, c);
        hand[i] = make_int2(row, c);
      }
      __syncthreads();
      if (wave == 0) {
        for (int g = i_lo / n; g <= i_hi / n; ++g) {
          const int i = g * n + lane;
          const bool act = lane < n && i >= i_lo && i <= i_hi;
          int row = 0, c = 0, k = 0;
          if (act) {
            const int2 hv = hand[i];
            row = hv.x;
            c = hv.y;
            const uint32_t* __restrict__ crow = a.cum + (size_t)row * CD_ROW;
            const uint32_t slot = x & (CD_TOTAL - 1u);
            k = CD_A;
            while (slot < crow[k]) --k;
            while (slot >= crow[k + 1]) ++k;
            const uint32_t cm = crow[k];
            x = (crow[k + 1] - cm) * (x >> CD_PREC) + slot - cm;
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
