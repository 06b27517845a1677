// Stockham FFT of power-of-two length L held in registers by a team of
// T = L/V threads (V = 16 values per thread for L = 1024, so that such a
// team is still one wavefront, 8 otherwise), with LDS exchanges between
// passes.
//
// Layout: on entry thread t of the team holds v[e] = X[t + e*T], e < V; on
// exit it holds v[e] = Xhat[t + e*T] in the same strided layout, so both the
// first pass's loads and the last pass's stores are unit-stride across the
// team (coalesced in global memory, conflict-free in LDS).
//
// Passes (self-sorting Stockham, decimation in time): one leading radix-2 or
// radix-4 pass when log2(L) is not a multiple of 3, then radix-8 passes.  A
// pass of radix R over span Ns treats butterflies j = t + u*T (u < V/R) with
// inputs X[j + r*L/R] = v[u + r*(V/R)], twiddles W_{Ns R}^{r k} (k = j mod
// Ns), an R-point DFT, and outputs at (j - k) R + k + r Ns.
//
// Pruning for the zero-padded Gram apply: HALF_IN declares X[i] = 0 for
// i >= L/2 (v[V/2..V-1] = 0 on entry, folded out of the first pass); a
// caller that only needs outputs i < L/2 reads only v[0..V/2-1], and the
// compiler drops the unused half of the last pass.
//
// Forward transform: Xhat[p] = sum_i X[i] exp(-2 pi i p / L); inverse: the
// conjugate kernel, unnormalised.
#pragma once
#include "common.hpp"

namespace recon {

template <int L>
struct FftShape {
  static constexpr int LOG = (L == 64) ? 6 : (L == 128) ? 7 : (L == 256) ? 8
                            : (L == 512) ? 9 : (L == 1024) ? 10 : (L == 2048) ? 11 : -1;
  static_assert(LOG > 0, "unsupported FFT length");
  static constexpr int V = (L == 1024) ? 16 : 8;  // values per thread
  static constexpr int T = L / V;                  // threads per team
  static constexpr int NR8 = LOG / 3;
  static constexpr int REM = LOG % 3;
  static constexpr int NP = NR8 + (REM ? 1 : 0);
  static constexpr int PAD = L + L / 8;  // padded LDS entries per buffer
  // Span of the first radix-8 pass that needs twiddles; the pass of span NS
  // finds W^{r k} (r = 1..7, k < NS) at tw[NS - S0 + (r - 1) NS + k].
  static constexpr int S0 = REM ? (1 << REM) : 8;
  static constexpr int TWN = L - S0;  // entries of the per-pass twiddle table
};

// LDS index padding: one spare slot every 8 entries breaks the stride-8
// write pattern of the first passes across banks.
__device__ __forceinline__ int lpad(int p) { return p + (p >> 3); }

// The transforms are written once for both element types: C = float2 (the
// FP32 iteration and the plain Gram apply) or double2 (the FP64 iteration).
template <bool INV, typename C>
__device__ __forceinline__ C mul_w4(C a) {  // a * exp(-+ 2 pi i / 4)
  return INV ? cmk<C>(-a.y, a.x) : cmk<C>(a.y, -a.x);
}
template <bool INV, typename C>
__device__ __forceinline__ C mul_w8(C a) {  // a * exp(-+ 2 pi i / 8)
  const real_t<C> s = (real_t<C>)0.70710678118654752440;
  return INV ? cmk<C>((a.x - a.y) * s, (a.x + a.y) * s)
             : cmk<C>((a.x + a.y) * s, (a.y - a.x) * s);
}
template <bool INV, typename C>
__device__ __forceinline__ C mul_w8_3(C a) {  // a * exp(-+ 2 pi i 3 / 8)
  const real_t<C> s = (real_t<C>)0.70710678118654752440;
  return INV ? cmk<C>((-a.x - a.y) * s, (a.x - a.y) * s)
             : cmk<C>((a.y - a.x) * s, (-a.x - a.y) * s);
}

// In-place R-point DFTs, natural order in and out.  HALF: a[R/2..R-1] = 0.
template <bool INV, bool HALF, typename C>
__device__ __forceinline__ void dft2(C* a) {
  if (HALF) {
    a[1] = a[0];
  } else {
    const C t = a[0];
    a[0] = c_add(t, a[1]);
    a[1] = c_sub(t, a[1]);
  }
}

template <bool INV, bool HALF, typename C>
__device__ __forceinline__ void dft4(C* a) {
  if (HALF) {
    const C w = mul_w4<INV>(a[1]);
    const C a0 = a[0], a1 = a[1];
    a[0] = c_add(a0, a1);
    a[2] = c_sub(a0, a1);
    a[1] = c_add(a0, w);
    a[3] = c_sub(a0, w);
  } else {
    const C s02 = c_add(a[0], a[2]), d02 = c_sub(a[0], a[2]);
    const C s13 = c_add(a[1], a[3]), d13 = mul_w4<INV>(c_sub(a[1], a[3]));
    a[0] = c_add(s02, s13);
    a[2] = c_sub(s02, s13);
    a[1] = c_add(d02, d13);
    a[3] = c_sub(d02, d13);
  }
}

template <bool INV, bool HALF, typename C>
__device__ __forceinline__ void dft8(C* a) {
  C e[4] = {a[0], a[2], a[4], a[6]};
  C o[4] = {a[1], a[3], a[5], a[7]};
  dft4<INV, HALF>(e);
  dft4<INV, HALF>(o);
  o[1] = mul_w8<INV>(o[1]);
  o[2] = mul_w4<INV>(o[2]);
  o[3] = mul_w8_3<INV>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = c_add(e[k], o[k]);
    a[k + 4] = c_sub(e[k], o[k]);
  }
}

template <int R, bool INV, bool HALF, typename C>
__device__ __forceinline__ void dft(C* a) {
  if constexpr (R == 2) dft2<INV, HALF>(a);
  else if constexpr (R == 4) dft4<INV, HALF>(a);
  else dft8<INV, HALF>(a);
}

// Twiddles of one thread kept in registers (for V = 8, one butterfly per
// radix-8 pass): the butterfly of pass P has a fixed k = t mod NS, and of its
// seven twiddles W^{rk} the ones for r = 1, 2, 4 are loaded from the plan's
// table g[i] = exp(-2 pi i i / L); r = 3, 5, 6, 7 are products of two of them
// (W^3 = W W^2, W^5 = W W^4, W^6 = W^2 W^4, W^7 = W^3 W^4: at most two
// roundings).  Loaded once, they serve every transform the thread runs.
template <int L, typename C>
struct TwRegs {
  using S = FftShape<L>;
  static_assert(S::V == 8, "one butterfly per radix-8 pass");
  static constexpr int NPT = S::NP - 1;  // passes with twiddles (P >= 1)
  C w[NPT > 0 ? NPT : 1][3];             // W^k, W^2k, W^4k
  __device__ __forceinline__ void load(const C* __restrict__ g, int t) {
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
      const int ns = S::S0 << (3 * p);  // span of pass p + 1
      const int k = t & (ns - 1);
      const int st = k * (L / (8 * ns));
      w[p][0] = g[st];
      w[p][1] = g[2 * st];
      w[p][2] = g[4 * st];
    }
  }
};

template <typename T>
struct IsTwRegs {
  static constexpr bool value = false;
};
template <int L, typename C>
struct IsTwRegs<TwRegs<L, C>> {
  static constexpr bool value = true;
};

// One twiddle per radix-8 pass and butterfly in registers: W^k of each of
// the thread's V/8 butterflies; the pass multiplies input r by W^{rk}, formed
// as the running product W^{(r-1)k} W^k, so that a single product is live at
// a time.  At V = 8 that needs a third of TwRegs' registers and none of the
// seven-entry array, at up to six roundings per power instead of two (used
// in FP64, where that is ~1e-15).
template <int L, typename C>
struct TwPow {
  using S = FftShape<L>;
  static constexpr int NPT = S::NP - 1;
  static constexpr int NB8 = S::V / 8;  // butterflies per radix-8 pass
  C w[NPT > 0 ? NPT : 1][NB8];
  __device__ __forceinline__ void load(const C* __restrict__ g, int t) {
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
      const int ns = S::S0 << (3 * p);  // span of pass p + 1
#pragma unroll
      for (int u = 0; u < NB8; ++u) w[p][u] = g[((t + u * S::T) & (ns - 1)) * (L / (8 * ns))];
    }
  }
};

template <typename T>
struct IsTwPow {
  static constexpr bool value = false;
};
template <int L, typename C>
struct IsTwPow<TwPow<L, C>> {
  static constexpr bool value = true;
};

// The seven twiddles W^{rk}, r = 1..7, of pass P from TwRegs.
template <int P, int L, typename C>
__device__ __forceinline__ void twiddles7(const TwRegs<L, C>& tw, C (&w)[7]) {
  const C w1 = tw.w[P - 1][0], w2 = tw.w[P - 1][1], w4 = tw.w[P - 1][2];
  w[0] = w1;
  w[1] = w2;
  w[2] = c_mul(w1, w2);
  w[3] = w4;
  w[4] = c_mul(w1, w4);
  w[5] = c_mul(w2, w4);
  w[6] = c_mul(w[2], w4);
}

// One Stockham pass (pass P, span NS); returns the output positions of v[e]
// in pos[e].
template <int L, int R, int NS, int P, bool INV, bool HALF, typename C, typename TW>
__device__ __forceinline__ void fft_pass(C (&v)[FftShape<L>::V], int t, const TW& tw,
                                         int (&pos)[FftShape<L>::V]) {
  constexpr int NB = FftShape<L>::V / R;
  constexpr int T = FftShape<L>::T;
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int j = t + u * T;
    const int k = j & (NS - 1);
    C a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[u + r * NB];
    if constexpr (NS > 1 && IsTwPow<TW>::value) {
      static_assert(R == 8, "twiddled passes are radix 8");
      C w1 = tw.w[P - 1][u];
      if (INV) w1.y = -w1.y;
      C w = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        a[r] = c_mul(a[r], w);
        if (r + 1 < R) w = c_mul(w, w1);
      }
    } else if constexpr (NS > 1 && IsTwRegs<TW>::value) {
      C w7[7];
      twiddles7<P>(tw, w7);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = w7[r - 1];
        if (INV) w.y = -w.y;
        a[r] = c_mul(a[r], w);
      }
    } else if constexpr (NS > 1) {
      // Per-pass LDS table: consecutive k are consecutive entries, so a
      // wave's twiddle reads are conflict-free (or broadcasts when NS < 64).
      constexpr int OFF = NS - FftShape<L>::S0;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tw[OFF + (r - 1) * NS + k];
        if (INV) w.y = -w.y;
        a[r] = c_mul(a[r], w);
      }
    }
    dft<R, INV, HALF>(a);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[u + r * NB] = a[r];
      pos[u + r * NB] = base + r * NS;
    }
  }
}

// Ordering of the LDS exchanges of a team.  A team that fits in one
// wavefront (L <= 512) needs no block barrier: LDS operations of a wave are
// performed in issue order, so a compiler-level fence between the writes and
// the reads of an exchange suffices, and one buffer can serve every pass.
// Larger teams span several waves and use block barriers with two buffers.
template <int L>
struct FftSync {
  static constexpr bool WAVE_LOCAL = FftShape<L>::T <= 64;
};

template <int L>
__device__ __forceinline__ void team_sync() {
  if constexpr (FftSync<L>::WAVE_LOCAL) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// LDS of one team's exchange buffers, in elements of C.  FP32 values are
// exchanged whole; FP64 values one component at a time (8-byte halves), so
// the buffer is half as large and the access pattern is the one of the FP32
// transform.  Multi-wave teams need two buffers (block barriers, no
// write-after-read wait between consecutive exchanges).
template <int L, typename C>
struct FftLds {
  static constexpr bool SPLIT = sizeof(C) == 16;
  static constexpr int BUFS = FftSync<L>::WAVE_LOCAL ? 1 : 2;
  static constexpr int TEAM = SPLIT ? BUFS * FftShape<L>::PAD / 2 : BUFS * FftShape<L>::PAD;
};

template <int L, typename C>
constexpr int fft_team_lds() {
  return FftLds<L, C>::TEAM;
}

// Exchange after pass P: value e goes to position pos[e] and comes back as
// element t + e*T.  tb: the team's buffers.
template <int L, int P, typename C>
__device__ __forceinline__ void fft_exchange(C (&v)[FftShape<L>::V],
                                             const int (&pos)[FftShape<L>::V], int t, C* tb) {
  using S = FftShape<L>;
  constexpr bool WL = FftSync<L>::WAVE_LOCAL;
  if constexpr (FftLds<L, C>::SPLIT) {
    double* b0 = reinterpret_cast<double*>(tb);
    double* b1 = b0 + (WL ? 0 : S::PAD);
#pragma unroll
    for (int e = 0; e < S::V; ++e) b0[lpad(pos[e])] = v[e].x;
    team_sync<L>();
#pragma unroll
    for (int e = 0; e < S::V; ++e) v[e].x = b0[lpad(t + e * S::T)];
    if constexpr (WL) team_sync<L>();  // reads before the writes of the other half
#pragma unroll
    for (int e = 0; e < S::V; ++e) b1[lpad(pos[e])] = v[e].y;
    team_sync<L>();
#pragma unroll
    for (int e = 0; e < S::V; ++e) v[e].y = b1[lpad(t + e * S::T)];
    if constexpr (WL) team_sync<L>();  // reads before the next writes
  } else {
    C* buf = (WL || !(P & 1)) ? tb : tb + S::PAD;
#pragma unroll
    for (int e = 0; e < S::V; ++e) buf[lpad(pos[e])] = v[e];
    team_sync<L>();
#pragma unroll
    for (int e = 0; e < S::V; ++e) v[e] = buf[lpad(t + e * S::T)];
    if constexpr (WL) team_sync<L>();  // reads before next writes
  }
}

template <int L, bool INV, bool HALF_IN, int P, int NS, typename C, typename TW>
__device__ __forceinline__ void fft_passes(C (&v)[FftShape<L>::V], int t, C* tb, const TW& tw) {
  using S = FftShape<L>;
  constexpr int R = (P == 0 && S::REM) ? (1 << S::REM) : 8;
  constexpr bool HALF = HALF_IN && (P == 0);
  int pos[S::V];
  fft_pass<L, R, NS, P, INV, HALF>(v, t, tw, pos);
  if constexpr (P + 1 < S::NP) {
    fft_exchange<L, P>(v, pos, t, tb);
    fft_passes<L, INV, HALF_IN, P + 1, NS * R>(v, t, tb, tw);
  }
  // Last pass: j < L/R = NS, so pos[e] = t + e*T and v is already in the
  // strided output layout.
}

// Full transform.  For L > 512 every thread of the block must call this
// (block barriers); for L <= 512 only the team's own wavefront is involved.
// tb: this team's exchange buffers (fft_team_lds<L, C>() elements of LDS);
// tw: the per-pass LDS twiddle table built by load_twiddles (a pointer), or
// the thread's TwRegs or TwPow.
template <int L, bool INV, bool HALF_IN, typename C, typename TW>
__device__ __forceinline__ void fft_team(C (&v)[FftShape<L>::V], int t, C* tb, const TW& tw) {
  if (HALF_IN) {
#pragma unroll
    for (int e = FftShape<L>::V / 2; e < FftShape<L>::V; ++e) v[e] = cmk<C>(0, 0);
  }
  fft_passes<L, INV, HALF_IN, 0, 1>(v, t, tb, tw);
}

// Build the per-pass twiddle table in LDS (TWN <= L entries) from the plan's
// table g[i] = exp(-2 pi i i / L): entry NS - S0 + (r - 1) NS + k of the pass
// of span NS holds g[r k L / (8 NS)].
template <int L, typename C>
__device__ __forceinline__ void load_twiddles(C* tw, const C* __restrict__ g) {
  using S = FftShape<L>;
  for (int i = threadIdx.x; i < S::TWN; i += blockDim.x) {
    int ns = S::S0;
#pragma unroll
    for (int p = 0; p < 3; ++p)
      if (i >= 8 * ns - S::S0) ns *= 8;
    const int q = i - (ns - S::S0);
    const int r = q / ns + 1, k = q - (r - 1) * ns;
    tw[i] = g[r * k * (L / (8 * ns))];
  }
}

}  // namespace recon
