// Teams of threads that hold one problem over an input of dimension n
// (a wave64 for n <= 1024, a 256-thread workgroup for n <= 4096), and the
// dispatch of (team, elements per member) from n.  Shared by the kernels that
// keep one subdomain's box in registers (relaxed and complete clipping).
#pragma once
#include "cv_common.h"

namespace {

constexpr int CV_TEAM_KMAX = 64;  // constraint slots whose metadata a team broadcasts

// A team of threads that holds one problem.  Wave: the 64 lanes of a wave,
// four problems per 256-thread workgroup, reductions by DPP and readlane,
// constraint metadata broadcast by readlane.  Block: the 256 threads of a
// workgroup, one problem each, reductions through LDS.  Every member calls
// every team operation (control flow is uniform within a team).
struct WaveTeam {
  static constexpr int SIZE = 64;
  static constexpr int PER_BLOCK = 4;
  int t;
  __device__ static int index_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
  __device__ double sum(double v) const { return wave_sum(v); }
  __device__ void sum3(double& a, double& b, double& c) const { wave_sum3(a, b, c); }
  __device__ double max(double v) const { return wave_max(v); }
  __device__ double min(double v) const { return wave_min(v); }
  // two maxima and a sum in one pass
  __device__ void max_max_sum(double& a, double& b, double& c) const {
    a = wave_max(a);
    b = wave_max(b);
    c = wave_sum(c);
  }
  // two sums and a maximum in one pass
  __device__ void sum_sum_max(double& a, double& b, double& c) const {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_max(c);
  }
  // member k < cnt holds constraint k's row pointer, scale and offset
  __device__ void publish(const float*, float, double, int) const {}
  __device__ void meta(const float* my_row, float my_scale, double my_h, int k, const float*& row,
                       float& scale, double& h) const {
    const uint64_t u = (uint64_t)(uintptr_t)my_row;
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, k);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), k);
    row = (const float*)(uintptr_t)(((uint64_t)hi << 32) | lo);
    scale = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_scale), k));
    h = lane_f64(my_h, k);
  }
};

struct BlockTeam {
  static constexpr int SIZE = 256;
  static constexpr int PER_BLOCK = 1;
  int t;
  double* red;          // LDS [24]: two banks of 12, used alternately
  const float** mrow;   // LDS [CV_TEAM_KMAX]
  float* mscale;        // LDS [CV_TEAM_KMAX]
  double* mh;           // LDS [CV_TEAM_KMAX]
  mutable int bank = 0;
  __device__ static int index_in_block() { return 0; }
  // One barrier per reduction: successive reductions write alternate banks,
  // and a thread reaching reduction i+1's barrier implies every thread has
  // read reduction i-1's bank (it wrote bank i first).
  __device__ double* next_bank() const {
    double* r = red + 12 * bank;
    bank ^= 1;
    return r;
  }
  __device__ double sum(double v) const {
    double* rb = next_bank();
    v = wave_sum(v);
    if ((t & 63) == 0) rb[t >> 6] = v;
    __syncthreads();
    return (rb[0] + rb[1]) + (rb[2] + rb[3]);
  }
  __device__ void sum3(double& a, double& b, double& c) const {
    double* rb = next_bank();
    wave_sum3(a, b, c);
    if ((t & 63) == 0) {
      rb[t >> 6] = a;
      rb[4 + (t >> 6)] = b;
      rb[8 + (t >> 6)] = c;
    }
    __syncthreads();
    a = (rb[0] + rb[1]) + (rb[2] + rb[3]);
    b = (rb[4] + rb[5]) + (rb[6] + rb[7]);
    c = (rb[8] + rb[9]) + (rb[10] + rb[11]);
  }
  __device__ double max(double v) const {
    double* rb = next_bank();
    v = wave_max(v);
    if ((t & 63) == 0) rb[t >> 6] = v;
    __syncthreads();
    return fmax(fmax(rb[0], rb[1]), fmax(rb[2], rb[3]));
  }
  // two maxima and a sum through one barrier (each combined as max, max
  // and sum would combine it)
  __device__ void max_max_sum(double& a, double& b, double& c) const {
    double* rb = next_bank();
    a = wave_max(a);
    b = wave_max(b);
    c = wave_sum(c);
    if ((t & 63) == 0) {
      rb[t >> 6] = a;
      rb[4 + (t >> 6)] = b;
      rb[8 + (t >> 6)] = c;
    }
    __syncthreads();
    a = fmax(fmax(rb[0], rb[1]), fmax(rb[2], rb[3]));
    b = fmax(fmax(rb[4], rb[5]), fmax(rb[6], rb[7]));
    c = (rb[8] + rb[9]) + (rb[10] + rb[11]);
  }
  // two sums and a maximum through one barrier
  __device__ void sum_sum_max(double& a, double& b, double& c) const {
    double* rb = next_bank();
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_max(c);
    if ((t & 63) == 0) {
      rb[t >> 6] = a;
      rb[4 + (t >> 6)] = b;
      rb[8 + (t >> 6)] = c;
    }
    __syncthreads();
    a = (rb[0] + rb[1]) + (rb[2] + rb[3]);
    b = (rb[4] + rb[5]) + (rb[6] + rb[7]);
    c = fmax(fmax(rb[8], rb[9]), fmax(rb[10], rb[11]));
  }
  __device__ double min(double v) const {
    double* rb = next_bank();
    v = wave_min(v);
    if ((t & 63) == 0) rb[t >> 6] = v;
    __syncthreads();
    return fmin(fmin(rb[0], rb[1]), fmin(rb[2], rb[3]));
  }
  __device__ void publish(const float* my_row, float my_scale, double my_h, int cnt) const {
    if (t < cnt) {
      mrow[t] = my_row;
      mscale[t] = my_scale;
      mh[t] = my_h;
    }
    __syncthreads();
  }
  // Every member reads the same LDS words, so the values are uniform: taking
  // them through readfirstlane puts them in scalar registers, which lets a
  // buffer load use the row as its resource directly (a resource the
  // compiler sees in vector registers costs a loop over its distinct values
  // around every load, each waiting for the previous).
  __device__ void meta(const float*, float, double, int k, const float*& row, float& scale,
                       double& h) const {
    row = uniform_ptr(mrow[k]);
    scale = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(mscale[k])));
    h = uniform_f64(mh[k]);
  }
};

// The team of member threadIdx.x, with its LDS scratch (used by BlockTeam).
template <class Team>
__device__ __forceinline__ Team make_team(double* red, const float** mrow, float* mscale,
                                          double* mh) {
  if constexpr (Team::PER_BLOCK == 1)
    return Team{(int)threadIdx.x, red, mrow, mscale, mh};
  else
    return Team{(int)(threadIdx.x & 63)};
}

int epl_for(int n) {
  const int e = (n + 63) / 64;
  if (e <= 1) return 1;
  if (e <= 2) return 2;
  if (e <= 4) return 4;
  if (e <= 8) return 8;
  if (e <= 13) return 13;
  if (e <= 16) return 16;
  return -1;
}

// Team TM and elements per member E for an input dimension n (<= 4096): a
// wave up to 1024 coordinates, a workgroup beyond.
#define CV_DISPATCH_TEAM(n, CALL)                                          \
  if ((n) <= 1024) {                                                       \
    typedef WaveTeam TM;                                                   \
    switch (epl_for(n)) {                                                  \
      case 1: { constexpr int E = 1; CALL; } break;                        \
      case 2: { constexpr int E = 2; CALL; } break;                        \
      case 4: { constexpr int E = 4; CALL; } break;                        \
      case 8: { constexpr int E = 8; CALL; } break;                        \
      case 13: { constexpr int E = 13; CALL; } break;                      \
      case 16: { constexpr int E = 16; CALL; } break;                      \
      default: return hipErrorInvalidValue;                                \
    }                                                                      \
  } else if ((n) <= 2048) {                                                \
    typedef BlockTeam TM; constexpr int E = 8; CALL;                       \
  } else if ((n) <= 3072) {                                                \
    typedef BlockTeam TM; constexpr int E = 12; CALL;                      \
  } else if ((n) <= 4096) {                                                \
    typedef BlockTeam TM; constexpr int E = 16; CALL;                      \
  } else {                                                                 \
    return hipErrorInvalidValue;                                           \
  }

inline unsigned team_blocks(long long problems, int per_block) {
  return (unsigned)((problems + per_block - 1) / per_block);
}

}  // namespace
