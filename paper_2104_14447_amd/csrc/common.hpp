// common.hpp -- shared device helpers of libgmls (gfx950, wave64).
//
// Compile-time tables of the eps-scaled Taylor basis (Section 2.1, basis
// equations): monomials of total degree <= m in graded order (within a degree,
// descending powers of x, then of y).  Every monomial but the constant has a
// parent with one power fewer, so p_a = p_parent * s_d / a_d evaluates the
// whole basis with one multiply per entry.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GMLS_WAVE 64

namespace gmls {

constexpr int binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int)r;
}

constexpr int num_mono(int dim, int deg) { return deg < 0 ? 0 : binom(deg + dim, dim); }

// Monomials of total degree <= DEG in DIM variables.
template <int DIM, int DEG>
struct Mono {
  static constexpr int N = num_mono(DIM, DEG);
  int e[N][3];
  int parent[N];  // index of the monomial with one power fewer in pdim
  int pdim[N];    // the variable removed
  int pexp[N];    // e[a][pdim[a]] (the divisor of the scaled basis)
  constexpr Mono() : e{}, parent{}, pdim{}, pexp{} {
    int q = 0;
    for (int deg = 0; deg <= DEG; ++deg) {
      if (DIM == 1) {
        e[q][0] = deg;
        ++q;
      } else if (DIM == 2) {
        for (int a = deg; a >= 0; --a) {
          e[q][0] = a;
          e[q][1] = deg - a;
          ++q;
        }
      } else {
        for (int a = deg; a >= 0; --a)
          for (int b = deg - a; b >= 0; --b) {
            e[q][0] = a;
            e[q][1] = b;
            e[q][2] = deg - a - b;
            ++q;
          }
      }
    }
    parent[0] = 0;
    pdim[0] = 0;
    pexp[0] = 1;
    for (int a = 1; a < N; ++a) {
      int d = 0;
      while (e[a][d] == 0) ++d;
      pdim[a] = d;
      pexp[a] = e[a][d];
      int want[3] = {e[a][0], e[a][1], e[a][2]};
      want[d] -= 1;
      for (int b = 0; b < N; ++b)
        if (e[b][0] == want[0] && e[b][1] == want[1] && e[b][2] == want[2]) parent[a] = b;
    }
  }
  constexpr int index(int a0, int a1, int a2) const {
    for (int b = 0; b < N; ++b)
      if (e[b][0] == a0 && e[b][1] == a1 && e[b][2] == a2) return b;
    return -1;
  }
};

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup i runs on
// XCD i % 8), and each XCD has its own L2.  This renumbering gives XCD x the
// contiguous logical range [x*nb/8, (x+1)*nb/8), so that neighbouring work
// items (spatially ordered targets) share one L2.  gridDim.x must be a
// multiple of 8.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// grid size rounded up to a multiple of the XCD count
inline int xcd_grid(int nb) { return nb < 8 ? 8 : (nb + 7) & ~7; }

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int2 b = __builtin_bit_cast(int2, v);
  b.x = __builtin_amdgcn_readlane(b.x, lane);
  b.y = __builtin_amdgcn_readlane(b.y, lane);
  return __builtin_bit_cast(double, b);
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ int readfirstlane_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int readlane_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// Wave-uniform copies (taken from the first active lane).  Every value that
// decides a branch or a loop exit of a whole wavefront goes through one of
// these, so that the compiler emits scalar branches: a branch it believes to
// be divergent is structurized with exec masks, and a lane-0 atomic followed
// by readfirstlane is then no longer guaranteed to see lane 0 active.
__device__ __forceinline__ double uniform_d(double v) {
  int2 b = __builtin_bit_cast(int2, v);
  b.x = __builtin_amdgcn_readfirstlane(b.x);
  b.y = __builtin_amdgcn_readfirstlane(b.y);
  return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  int2 b = __builtin_bit_cast(int2, v);
  b.x = __builtin_amdgcn_readfirstlane(b.x);
  b.y = __builtin_amdgcn_readfirstlane(b.y);
  return __builtin_bit_cast(int64_t, b);
}

// v from the lane selected by a DPP control word (both halves of a double)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int2 b = __builtin_bit_cast(int2, v);
  b.x = __builtin_amdgcn_update_dpp(0, b.x, CTRL, 0xF, 0xF, false);
  b.y = __builtin_amdgcn_update_dpp(0, b.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, b);
}

// v[lane] + v[lane ^ 16] (S = 16) or v[lane] + v[lane ^ 32] (S = 32) by the
// lane-swap instructions: swapping the odd 16-lane rows (the upper half) of
// one copy of v with the even rows (lower half) of another leaves the lower
// partner in the first copy and the upper one in the second, in every lane,
// so both lanes of a pair add the same operands in the same order.
template <int S>
__device__ __forceinline__ double swap_pair_sum(double v) {
  static_assert(S == 16 || S == 32, "row or half swap");
  const int2 b = __builtin_bit_cast(int2, v);
  int2 lo, hi;
  if constexpr (S == 16) {
    const auto x = __builtin_amdgcn_permlane16_swap(b.x, b.x, false, false);
    const auto y = __builtin_amdgcn_permlane16_swap(b.y, b.y, false, false);
    lo = make_int2(x[0], y[0]);
    hi = make_int2(x[1], y[1]);
  } else {
    const auto x = __builtin_amdgcn_permlane32_swap(b.x, b.x, false, false);
    const auto y = __builtin_amdgcn_permlane32_swap(b.y, b.y, false, false);
    lo = make_int2(x[0], y[0]);
    hi = make_int2(x[1], y[1]);
  }
  return __builtin_bit_cast(double, lo) + __builtin_bit_cast(double, hi);
}

// Sum of v over all 64 lanes, bitwise the same in every lane, with no LDS
// traffic and no scalar reads: within each 16-lane row by DPP (swap
// neighbours, swap pairs, mirror the row, rotate by 8: at every step the two
// lanes that combine add the same two operands, so the row sum is identical
// across the row), then rows 0 + 1 and 2 + 3, then the two halves, by lane
// swaps.  Every lane must be active.
__device__ __forceinline__ double wave_sum_uniform(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x140>(v);  // row_mirror
  v += dpp_d<0x128>(v);  // row_ror:8
  return swap_pair_sum<32>(swap_pair_sum<16>(v));
}

// LDS writes of one wavefront are seen by its later LDS reads from any lane
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

// sum over the G consecutive lanes of a group (G a power of two <= 64)
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

template <int G, typename T>
__device__ __forceinline__ T group_max(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, G);
    v = o > v ? o : v;
  }
  return v;
}

// exclusive prefix count of `pred` over the lanes below this one
__device__ __forceinline__ int ballot_prefix(bool pred, uint64_t *mask_out) {
  uint64_t m = __ballot(pred);
  *mask_out = m;
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ double int_pow(double b, int p) {
  double r = 1.0;
  for (int q = 0; q < p; ++q) r *= b;
  return r;
}

}  // namespace gmls
