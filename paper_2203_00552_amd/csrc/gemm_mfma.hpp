// Dense products against the shared harmonic tables on the FP64 matrix cores.
//
// Two transforms of every sphere's data go through the same fixed table (Sec. 2.2):
//   synthesis  zr[k][n] = sum_l Z[k][l] Y_l(s_n)            (coefficients -> grid values)
//   projection out[k][l] = sum_n V[k][n] w_n Y_l(s_n)        (grid values -> coefficients)
// for the 2M rows k (two parts per sphere).  Both are out = A B (+ c0 base) with A the
// per-sphere rows (streamed once from HBM) and B the table (N x L doubles, shared by
// every row and read from the L2), so they are dense contractions of depth L or N and
// run here as v_mfma_f64_16x16x4 tiles.
//
// Layout of one launch: a block takes a chunk of 16 S rows of A, stages it in LDS
// (coalesced, zero-padded to a multiple of four in the depth and to an odd row stride
// against bank conflicts), and each of its wavefronts walks the 16-column tiles of the
// output assigned to it.  For a tile, the wavefront walks the depth four at a time:
// one load of a 4 x 16 fragment of B (16 consecutive doubles per row of the fragment,
// issued eight steps ahead), then S matrix operations, one per 16-row strip of the chunk, into S independent
// accumulators.  Each result element is the same fixed-order sum in every launch.
//
// Operand layout of v_mfma_f64_16x16x4f64 (64 lanes, lane = i + 16 q):
//   A fragment (16 x 4): lane holds A[i][q];  B fragment (4 x 16): lane holds B[q][i];
//   result (16 x 16), four doubles per lane: element r is D[q + 4 r][i] (measured on
//   gfx950 with unit fragments).
#pragma once
#include <hip/hip_runtime.h>

namespace ddlpb {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kGemmWaves = 8;  // wavefronts per block (at most)
constexpr int kPf = 8;         // steps of the B fragment fetched ahead

// out[r][c] = sum_k A[r][k] B[k][c] (+ c0 base[r][c] if base), r < R, c < C, k < K.
// A row-major with leading dimension lda; B row-major [K][ldb]; out and base row-major
// with leading dimension ldo (base may equal out).  Rows of a chunk are 16 S; the LDS
// holds 16 S x ap doubles, ap = 4 ceil(K / 4) + 1.
template <int S>
__global__ __launch_bounds__(64 * kGemmWaves) void k_gemm_f64(int R, int C, int K, const double* __restrict__ A,
                                                              int lda, const double* __restrict__ B, int ldb,
                                                              const double* base, double c0, double* out, int ldo) {
  extern __shared__ double as[];
  const int ks = (K + 3) >> 2, ap = 4 * ks + 1;
  const long r0 = (long)blockIdx.x * (16 * S);
  const int rows = (int)min((long)(16 * S), (long)R - r0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // stage the chunk: one row per wavefront at a time, zeros past K and past the last row
  for (int rr = w; rr < 16 * S; rr += nw) {
    const double* __restrict__ src = A + (r0 + rr) * lda;
    for (int kk = lane; kk < ap; kk += 64) as[rr * ap + kk] = (rr < rows && kk < K) ? src[kk] : 0.0;
  }
  __syncthreads();
  const int i = lane & 15, q = lane >> 4;
  const int ct = (C + 15) >> 4;
  for (int t = w; t < ct; t += nw) {
    const int col = 16 * t + i;
    const bool cok = col < C;
    dbl4 acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = dbl4{0.0, 0.0, 0.0, 0.0};
    // B fragment of step k: B[4 k + q][col], fetched kPf steps ahead into a ring of
    // registers (the table comes from the L2: several loads stay in flight per wave)
    double bq[kPf];
#pragma unroll
    for (int p = 0; p < kPf; ++p) {
      const int kb = 4 * p + q;
      bq[p] = (cok && kb < K) ? B[(long)kb * ldb + col] : 0.0;
    }
    for (int k0 = 0; k0 < ks; k0 += kPf) {
#pragma unroll
      for (int p = 0; p < kPf; ++p) {
        const int k = k0 + p;
        if (k < ks) {
          const double b = bq[p];
          const int kb = 4 * (k + kPf) + q;
          bq[p] = (cok && kb < K) ? B[(long)kb * ldb + col] : 0.0;
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const double a = as[(16 * s + i) * ap + 4 * k + q];
            acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
          }
        }
      }
    }
    if (cok) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int rr = 16 * s + q + 4 * e;
          if (rr < rows) {
            const long o = (r0 + rr) * ldo + col;
            out[o] = base ? fma(c0, base[o], acc[s][e]) : acc[s][e];
          }
        }
      }
    }
  }
}

// The same product for C <= 16 kGemmWaves (one 16-column tile per wavefront) and a
// deep contraction: the block walks the depth in chunks of KC (a multiple of 4), so that
// its LDS chunk (16 S x (KC + 1) doubles) stays small and several blocks share a
// compute unit; the accumulators persist across the chunks.
template <int S>
__global__ __launch_bounds__(64 * kGemmWaves) void k_gemm_f64_kc(int R, int C, int K, int KC,
                                                                 const double* __restrict__ A, int lda,
                                                                 const double* __restrict__ B, int ldb,
                                                                 const double* base, double c0, double* out,
                                                                 int ldo) {
  extern __shared__ double as[];
  const int ap = KC + 1;
  const long r0 = (long)blockIdx.x * (16 * S);
  const int rows = (int)min((long)(16 * S), (long)R - r0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int col = 16 * w + i;
  const bool cok = col < C;
  dbl4 acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();  // the previous chunk is consumed
    for (int rr = w; rr < 16 * S; rr += nw) {
      const double* __restrict__ src = A + (r0 + rr) * lda + k0;
      for (int kk = lane; kk < KC; kk += 64) as[rr * ap + kk] = (rr < rows && k0 + kk < K) ? src[kk] : 0.0;
    }
    __syncthreads();
    const int ks = min(KC, K - k0 + 3) >> 2;  // steps of four in this chunk
    double bq[kPf];
#pragma unroll
    for (int p = 0; p < kPf; ++p) {
      const int kb = k0 + 4 * p + q;
      bq[p] = (cok && p < ks && kb < K) ? B[(long)kb * ldb + col] : 0.0;
    }
    for (int kq = 0; kq < ks; kq += kPf) {
#pragma unroll
      for (int p = 0; p < kPf; ++p) {
        const int k = kq + p;
        if (k < ks) {
          const double b = bq[p];
          const int kb = k0 + 4 * (k + kPf) + q;
          bq[p] = (cok && k + kPf < ks && kb < K) ? B[(long)kb * ldb + col] : 0.0;
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const double a = as[(16 * s + i) * ap + 4 * k + q];
            acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
          }
        }
      }
    }
  }
  if (cok) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = 16 * s + q + 4 * e;
        if (rr < rows) {
          const long o = (r0 + rr) * ldo + col;
          out[o] = base ? fma(c0, base[o], acc[s][e]) : acc[s][e];
        }
      }
    }
  }
}

// LDS bytes of a launch with S strips per chunk
inline size_t gemm_f64_lds(int S, int K) { return (size_t)16 * S * (4 * ((K + 3) / 4) + 1) * sizeof(double); }

}  // namespace ddlpb
