// Register-blocked Stockham FFT for one line held by a team of T threads.
//
// A line of N complex points is spread over T = N / P threads, thread t
// holding x[t + T*m], m = 0..P-1 ("strided layout").  Each radix-R stage runs
// P/R butterflies per thread entirely in registers; between stages the line
// is exchanged through LDS (interleaved complex, padded to spread banks).  The Stockham autosort ordering makes the first
// stage read and the last stage write the strided layout directly, so a
// transform costs (#stages - 1) LDS round trips and the result of X[k]
// lands on thread k % T, register k / T -- natural order, coalesced for
// global stores.
//
// DIR = -1: X[k] = sum_n x[n] e^{-2 pi i nk/N};  DIR = +1: the unscaled inverse.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rift2 {

// Twiddle tables, one per supported line length, concatenated: entry
// tw_offset(N) + m holds e^{-2 pi i m / N}.  A length's table is contiguous,
// so the twiddles one stage reads share cache lines.
constexpr int kTwLengths[] = {256, 512, 768, 1024, 1536, 2048, 4096};
__host__ __device__ constexpr int tw_offset(int n) {
  int off = 0;
  for (int len : kTwLengths) {
    if (len == n) return off;
    off += len;
  }
  return -1;
}
constexpr int kTwTotal = 256 + 512 + 768 + 1024 + 1536 + 2048 + 4096;
__device__ float2 g_twiddle[kTwTotal];

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// a * e^{DIR i pi/2}
template <int DIR>
__device__ __forceinline__ float2 mul_quarter(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// cos(2 pi m / 16) for m = 0..15
__host__ __device__ constexpr float cos16(int m) {
  return (m & 15) == 0 ? 1.0f
       : (m & 15) == 1 ? 0.92387953251128674f
       : (m & 15) == 2 ? 0.70710678118654752f
       : (m & 15) == 3 ? 0.38268343236508977f
       : (m & 15) == 4 ? 0.0f
       : (m & 15) == 5 ? -0.38268343236508977f
       : (m & 15) == 6 ? -0.70710678118654752f
       : (m & 15) == 7 ? -0.92387953251128674f
       : (m & 15) == 8 ? -1.0f
       : (m & 15) == 9 ? -0.92387953251128674f
       : (m & 15) == 10 ? -0.70710678118654752f
       : (m & 15) == 11 ? -0.38268343236508977f
       : (m & 15) == 12 ? 0.0f
       : (m & 15) == 13 ? 0.38268343236508977f
       : (m & 15) == 14 ? 0.70710678118654752f
                        : 0.92387953251128674f;
}

// a * e^{DIR 2 pi i M / 16}, trivial angles without multiplications
template <int DIR, int M>
__device__ __forceinline__ float2 rot16(float2 a) {
  constexpr int m = M & 15;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return mul_quarter<DIR>(a);
  } else if constexpr (m == 8) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (m == 12) {
    return mul_quarter<-DIR>(a);
  } else {
    constexpr float c = cos16(m);
    constexpr float s = DIR * cos16(m + 12);  // DIR * sin(2 pi m / 16)
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
  const float2 t2 = cadd(x1, x3), t3 = mul_quarter<DIR>(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

template <int DIR>
__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
  constexpr float kS3 = 0.86602540378443865f;  // sqrt(3)/2
  const float2 t1 = cadd(b, c);
  const float2 t2 = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
  const float2 d = csub(b, c);
  // DIR * i * sqrt(3)/2 * (b - c)
  const float2 t3 = DIR < 0 ? make_float2(kS3 * d.y, -kS3 * d.x) : make_float2(-kS3 * d.y, kS3 * d.x);
  a = cadd(a, t1);
  b = cadd(t2, t3);
  c = csub(t2, t3);
}

// In-register R-point DFT in natural order (R in {2, 3, 4, 8, 16}).
template <int DIR, int R>
__device__ __forceinline__ void dft(float2 (&u)[R]) {
  if constexpr (R == 2) {
    dft2<DIR>(u[0], u[1]);
  } else if constexpr (R == 3) {
    dft3<DIR>(u[0], u[1], u[2]);
  } else if constexpr (R == 4) {
    dft4<DIR>(u[0], u[1], u[2], u[3]);
  } else if constexpr (R == 8) {
    // n = 2 n1 + n2: DFT4 over n1, twiddle w8^(n2 k1), DFT2 over n2 -> X[k1 + 4 k2]
    dft4<DIR>(u[0], u[2], u[4], u[6]);
    dft4<DIR>(u[1], u[3], u[5], u[7]);
    const float2 a0 = u[0], a1 = u[2], a2 = u[4], a3 = u[6];
    const float2 b0 = u[1], b1 = rot16<DIR, 2>(u[3]), b2 = rot16<DIR, 4>(u[5]), b3 = rot16<DIR, 6>(u[7]);
    u[0] = cadd(a0, b0);
    u[4] = csub(a0, b0);
    u[1] = cadd(a1, b1);
    u[5] = csub(a1, b1);
    u[2] = cadd(a2, b2);
    u[6] = csub(a2, b2);
    u[3] = cadd(a3, b3);
    u[7] = csub(a3, b3);
  } else if constexpr (R == 16) {
    // n = 4 n1 + n2: DFT4 over n1 (k1), twiddle w16^(n2 k1), DFT4 over n2 (k2) -> X[k1 + 4 k2]
    dft4<DIR>(u[0], u[4], u[8], u[12]);
    dft4<DIR>(u[1], u[5], u[9], u[13]);
    dft4<DIR>(u[2], u[6], u[10], u[14]);
    dft4<DIR>(u[3], u[7], u[11], u[15]);
    // a[n2][k1] = u[n2 + 4 k1]
    float2 c0[4] = {u[0], u[1], rot16<DIR, 0>(u[2]), u[3]};
    float2 c1[4] = {u[4], rot16<DIR, 1>(u[5]), rot16<DIR, 2>(u[6]), rot16<DIR, 3>(u[7])};
    float2 c2[4] = {u[8], rot16<DIR, 2>(u[9]), rot16<DIR, 4>(u[10]), rot16<DIR, 6>(u[11])};
    float2 c3[4] = {u[12], rot16<DIR, 3>(u[13]), rot16<DIR, 6>(u[14]), rot16<DIR, 9>(u[15])};
    dft4<DIR>(c0[0], c0[1], c0[2], c0[3]);
    dft4<DIR>(c1[0], c1[1], c1[2], c1[3]);
    dft4<DIR>(c2[0], c2[1], c2[2], c2[3]);
    dft4<DIR>(c3[0], c3[1], c3[2], c3[3]);
    // c_{k1}[k2] -> X[k1 + 4 k2]
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      u[0 + 4 * k2] = c0[k2];
      u[1 + 4 * k2] = c1[k2];
      u[2 + 4 * k2] = c2[k2];
      u[3 + 4 * k2] = c3[k2];
    }
  }
}

// Radix plans: N = product of radices, every radix divides P.
template <int N, int P>
struct FftPlan;

#define RIFT2_PLAN(N_, P_, NR_, R0, R1, R2, R3, R4, R5)                          \
  template <>                                                                  \
  struct FftPlan<N_, P_> {                                                     \
    static constexpr int N = N_, P = P_, T = N_ / P_, NR = NR_;                \
    static constexpr int rad(int i) {                                          \
      return i == 0 ? R0 : i == 1 ? R1 : i == 2 ? R2 : i == 3 ? R3 : i == 4 ? R4 : R5; \
    }                                                                          \
  };

RIFT2_PLAN(256, 16, 2, 16, 16, 1, 1, 1, 1)
RIFT2_PLAN(512, 16, 3, 16, 16, 2, 1, 1, 1)
RIFT2_PLAN(1024, 16, 3, 16, 16, 4, 1, 1, 1)
RIFT2_PLAN(2048, 16, 3, 16, 16, 8, 1, 1, 1)
RIFT2_PLAN(4096, 16, 3, 16, 16, 16, 1, 1, 1)
RIFT2_PLAN(768, 12, 5, 4, 4, 4, 4, 3, 1)
RIFT2_PLAN(1536, 12, 6, 4, 4, 4, 4, 2, 3)
RIFT2_PLAN(256, 4, 4, 4, 4, 4, 4, 1, 1)
RIFT2_PLAN(512, 8, 3, 8, 8, 8, 1, 1, 1)
RIFT2_PLAN(1024, 8, 4, 8, 8, 8, 2, 1, 1)
RIFT2_PLAN(2048, 8, 4, 8, 8, 8, 4, 1, 1)
#undef RIFT2_PLAN

// LDS lines hold interleaved complex values (one float2 per point).  The
// padded index puts one spare point after every 16 so radix-16 strides do not
// land on one bank.  When L consecutive lanes of a wave work on one line and
// the next L lanes on the next line, lines are L points apart modulo 32 so
// that neighbouring lines start on different banks.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
template <int N, int L = 32>
constexpr int lds_line() {
  return ((N + N / 16 + 31) / 32) * 32 + (L % 32);
}

// Buffer resource word 3 for raw (untyped) buffer access on gfx9.
constexpr int kRawBufferWord3 = 0x00020000;

// Twiddle e^{DIR 2 pi i m / N}, 0 <= m < N.
template <int DIR, int N>
__device__ __forceinline__ float2 twiddle(uint32_t m) {
  static_assert(tw_offset(N) >= 0, "no twiddle table for this length");
  // A raw buffer load: the table's base and length sit in a scalar resource
  // and each lane supplies a 32-bit byte offset, so a hoisted offset costs no
  // per-use address arithmetic (reads past the table would return zero).
  // The scalar offset is opaque so the load itself stays inside the loop
  // that uses it: hoisting every stage's twiddles out of the filter loops
  // costs more registers than the reloads.
  const __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)(g_twiddle + tw_offset(N)), 0, N * (int)sizeof(float2), kRawBufferWord3);
  int soff = 0;
  asm volatile("" : "+s"(soff));
  float2 w = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rsrc, m * (uint32_t)sizeof(float2), soff, 0));
  if (DIR > 0) w.y = -w.y;
  return w;
}

template <int DIR, int N, int T, int P, int R, int NS>
__device__ __forceinline__ void fft_stage(float2 (&v)[P], int t) {
  constexpr int NB = P / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    float2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[b + r * NB];
    if constexpr (NS > 1) {
      const uint32_t jm = (uint32_t)(t + T * b) % NS;
      constexpr uint32_t step = N / (NS * R);
#pragma unroll
      for (int r = 1; r < R; ++r) u[r] = cmul(u[r], twiddle<DIR, N>(r * jm * step));
    }
    dft<DIR, R>(u);
#pragma unroll
    for (int r = 0; r < R; ++r) v[b + r * NB] = u[r];
  }
}

// Orders this wave's LDS accesses before and after it (lanes of one wave
// exchange data through LDS without a block barrier; the LDS serves one
// wave's requests in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Team synchronisation: a block barrier, or a wave barrier when the team is
// one wave (T = 64) and nobody else touches its line.
template <bool WAVE>
__device__ __forceinline__ void team_sync() {
  if constexpr (WAVE) {
    wave_sync();
  } else {
    __syncthreads();
  }
}

// Write stage outputs to their Stockham positions, read back the strided layout.
template <int N, int T, int P, int R, int NS, bool WAVE>
__device__ __forceinline__ void fft_exchange(float2 (&v)[P], int t, float2* line) {
  constexpr int NB = P / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + T * b;
    const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) line[lds_pad(base + r * NS)] = v[b + r * NB];
  }
  team_sync<WAVE>();
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = line[lds_pad(t + T * m)];
  team_sync<WAVE>();
}

template <int DIR, class PL, int S, int NS, bool WAVE>
__device__ __forceinline__ void fft_run(float2 (&v)[PL::P], int t, float2* line) {
  if constexpr (S < PL::NR) {
    constexpr int R = PL::rad(S);
    fft_stage<DIR, PL::N, PL::T, PL::P, R, NS>(v, t);
    if constexpr (S + 1 < PL::NR) {
      fft_exchange<PL::N, PL::T, PL::P, R, NS, WAVE>(v, t, line);
      fft_run<DIR, PL, S + 1, NS * R, WAVE>(v, t, line);
    }
  }
}

// Two lines of one team transformed together: each stage's butterflies of
// both lines (twiddles read once), then one exchange for both, so the lines
// share every barrier and the wave has two independent chains to issue.
template <int DIR, int N, int T, int P, int R, int NS>
__device__ __forceinline__ void fft_stage2(float2 (&v0)[P], float2 (&v1)[P], int t) {
  constexpr int NB = P / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    float2 u0[R], u1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      u0[r] = v0[b + r * NB];
      u1[r] = v1[b + r * NB];
    }
    if constexpr (NS > 1) {
      const uint32_t jm = (uint32_t)(t + T * b) % NS;
      constexpr uint32_t step = N / (NS * R);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = twiddle<DIR, N>(r * jm * step);
        u0[r] = cmul(u0[r], w);
        u1[r] = cmul(u1[r], w);
      }
    }
    dft<DIR, R>(u0);
    dft<DIR, R>(u1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v0[b + r * NB] = u0[r];
      v1[b + r * NB] = u1[r];
    }
  }
}

template <int N, int T, int P, int R, int NS, bool WAVE>
__device__ __forceinline__ void fft_exchange2(float2 (&v0)[P], float2 (&v1)[P], int t, float2* l0, float2* l1) {
  constexpr int NB = P / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + T * b;
    const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      l0[lds_pad(base + r * NS)] = v0[b + r * NB];
      l1[lds_pad(base + r * NS)] = v1[b + r * NB];
    }
  }
  team_sync<WAVE>();
#pragma unroll
  for (int m = 0; m < P; ++m) {
    v0[m] = l0[lds_pad(t + T * m)];
    v1[m] = l1[lds_pad(t + T * m)];
  }
  team_sync<WAVE>();
}

template <int DIR, class PL, int S, int NS, bool WAVE>
__device__ __forceinline__ void fft_run2(float2 (&v0)[PL::P], float2 (&v1)[PL::P], int t, float2* l0, float2* l1) {
  if constexpr (S < PL::NR) {
    constexpr int R = PL::rad(S);
    fft_stage2<DIR, PL::N, PL::T, PL::P, R, NS>(v0, v1, t);
    if constexpr (S + 1 < PL::NR) {
      fft_exchange2<PL::N, PL::T, PL::P, R, NS, WAVE>(v0, v1, t, l0, l1);
      fft_run2<DIR, PL, S + 1, NS * R, WAVE>(v0, v1, t, l0, l1);
    }
  }
}

// Two lines of one team (each with its own LDS line of lds_line<N>() points);
// the same contract as fft_line otherwise.
template <int DIR, int N, int P, bool WAVE = false>
__device__ __forceinline__ void fft_line2(float2 (&v0)[P], float2 (&v1)[P], int t, float2* l0, float2* l1) {
  static_assert(!WAVE || N / P == 64, "a wave team is 64 threads");
  fft_run2<DIR, FftPlan<N, P>, 0, 1, WAVE>(v0, v1, t, l0, l1);
}

// Transform one line in the strided layout; `line` is this team's LDS line of
// lds_line<N>() points.  With WAVE = false every thread of the block must
// call this (it contains block barriers); with WAVE = true the team is one
// whole wave (T = 64) that owns `line` alone, and no block barrier is used.
template <int DIR, int N, int P, bool WAVE = false>
__device__ __forceinline__ void fft_line(float2 (&v)[P], int t, float2* line) {
  static_assert(!WAVE || N / P == 64, "a wave team is 64 threads");
  fft_run<DIR, FftPlan<N, P>, 0, 1, WAVE>(v, t, line);
}

}  // namespace rift2
