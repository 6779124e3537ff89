// GMRES-SDR device kernels for gfx950 (wave64, LDS-staged sketches).
//
// Per Arnoldi step j (Algorithm 1, truncated Arnoldi with one sketch per step):
//   stream A (the Arnoldi chain)
//     k_spmv_dia_sketch / k_spmv_sketch (matrix by diagonals / CSR)
//                    w = A p_{j-1}, partial window products <p_i, w>, ||w||^2,
//                    and the sketch S p_{j-1} with ||p_{j-1}||^2: the SpMV reads
//                    p_{j-1} anyway, so the one sketch per step costs no
//                    extra pass over HBM
//     k_update       reduces the window products and ||p_{j-1}||^2 in its
//                    prologue, then p_j = (w - sum c_i p_i) / nu_{j-1} in place
//   stream B (the sketched least squares, a chunk of steps per launch, behind
//   the event of the SpMV that completes the chunk's last sketch)
//     k_reduce_steps fixed-order reduction of the chunk's partial slots
//     k_lsq_steps_reg H column, SV and SAV columns, QR append, sketched
//                    residual, step record and halt, step after step with
//                    the Q factor held in registers
// Stored basis vectors are p_j = H(j+1, j) v_j: the orthogonalised A v_{j-1},
// so nu_j = ||p_j|| = H(j+1, j) stays of the order of ||A|| in every
// precision; the norms are folded into the coefficients, which saves a
// normalisation pass per step.

#include <hip/hip_ext.h>

#include <algorithm>

#include "sdr_kernels.h"

namespace sdr {

// ------------------------------------------------------------ reductions --
// Lane exchange within rows of 16 lanes by DPP (a VALU modifier, no LDS
// round trip): CTRL 0xB1 / 0x4E swap neighbours / pairs inside each quad,
// 0x124 / 0x128 rotate each row by 4 / 8 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the 64 lanes of a wave (all lanes active); the same value in every
// lane and the same bits on every call.  Row sums by DPP, then the four rows.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x124>(v);
  v += dpp_mov<0x128>(v);
  return (read_lane(v, 15) + read_lane(v, 31)) + (read_lane(v, 47) + read_lane(v, 63));
}
__device__ __forceinline__ cx<double> wave_sum(cx<double> v) { return {wave_sum(v.x), wave_sum(v.y)}; }

// Sums over the 64 lanes of NC per-lane values d[c] (NC = 8, 16 or 32); every
// lane gets every sum, the same bits on every call.  Quads first (DPP), then
// the 16 quad sums of each value are transposed through this wave's LDS
// scratch (16 x (NC + 1) doubles, odd pitch: no bank conflicts), each of
// G = 64 / NC consecutive lanes adds 16 / G of them, a DPP step combines the
// G lanes and readlane broadcasts.  One pass for all NC values instead of NC
// separate reductions.
template <int NC>
__device__ __forceinline__ void wave_sums(double (&d)[NC], double* scr) {
  static_assert(NC == 8 || NC == 16 || NC == 32, "NC");
  constexpr int P = NC + 1, G = 64 / NC, PER = 16 / G;
  const int lane = threadIdx.x & 63, quad = lane >> 2, sub = lane & 3;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    d[c] += dpp_mov<0xB1>(d[c]);
    d[c] += dpp_mov<0x4E>(d[c]);
  }
  // lane (quad, sub) stores values c = sub, sub + 4, ... of its quad
#pragma unroll
  for (int c = 0; c < NC; c += 4) {
    double v = d[c];
#pragma unroll
    for (int k = 1; k < 4; ++k)
      if (sub == k) v = d[c + k];
    scr[quad * P + c + sub] = v;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int col = lane / G, part = lane % G;
  double t = scr[(part * PER) * P + col];
#pragma unroll
  for (int i = 1; i < PER; ++i) t += scr[(part * PER + i) * P + col];
  if (G >= 2) t += dpp_mov<0xB1>(t);
  if (G >= 4) t += dpp_mov<0x4E>(t);
#pragma unroll
  for (int c = 0; c < NC; ++c)
    d[c] = G == 8 ? read_lane(t, G * c) + read_lane(t, G * c + 4) : read_lane(t, G * c);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void split_re(double v, double* o) { o[0] = v; }
__device__ __forceinline__ void split_re(cx<double> v, double* o) { o[0] = v.x; o[1] = v.y; }
__device__ __forceinline__ void join_re(double& v, const double* o) { v = o[0]; }
__device__ __forceinline__ void join_re(cx<double>& v, const double* o) { v = cx<double>{o[0], o[1]}; }
template <class A> struct ncomp { static constexpr int v = 1; };
template <> struct ncomp<cx<double>> { static constexpr int v = 2; };

// Sum of one value per thread over the block, same order on every call.
// red must hold blockDim.x / 64 entries; result valid in every thread.
template <class A>
__device__ A block_sum(A v, A* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  A s = red[0];
  for (int i = 1; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_add(cx<double>* p, cx<double> v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}

__device__ __forceinline__ double neg_if(double v, bool n) { return n ? -v : v; }
__device__ __forceinline__ cx<double> neg_if(cx<double> v, bool n) { return n ? -v : v; }

// Scatter one element's value into the zeta rows of S's column `col`.
template <class A>
__device__ __forceinline__ void sketch_word(A* acc, uint64_t h, int g, A v, const SketchSpec& sk) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = 4 * g + q;
    if (b < sk.zeta) {
      const uint32_t u = (uint32_t)(h >> (16 * q)) & 0xFFFFu;
      const int row = b * sk.bsz + (int)(((u >> 1) * (uint32_t)sk.bsz) >> 15);
      lds_add(&acc[row], neg_if(v, (u & 1u) != 0u));
    }
  }
}

template <class A>
__device__ __forceinline__ void sketch_scatter(A* acc, int64_t col, A v, const SketchSpec& sk) {
  const uint64_t base = sk.seed + kGamma * ((uint64_t)col * (uint64_t)sk.words + 1ull);
  if (sk.words <= 2) {  // zeta <= 8: both words unrolled
    sketch_word(acc, mix64(base), 0, v, sk);
    if (sk.words == 2) sketch_word(acc, mix64(base + kGamma), 1, v, sk);
  } else {
    for (int g = 0; g < sk.words; ++g) sketch_word(acc, mix64(base + (uint64_t)g * kGamma), g, v, sk);
  }
}

// Column sum of a [ncols x nb] partial array in the order every reducer of
// this library uses (thread-strided, then the fixed block tree), so that the
// same partials always give the same bits.
// Loads go out four at a time (indices clamped into range, so none sits
// behind a branch) and are added in index order.
template <class A>
__device__ __forceinline__ A col_sum(const A* __restrict__ part, int nb, int col, A* red) {
  const A* p = part + (int64_t)col * nb;
  A sum = zero<A>();
  for (int i0 = threadIdx.x; i0 < nb; i0 += 4 * kBlock) {
    A v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = p[min(i0 + u * kBlock, nb - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * kBlock < nb) sum += v[u];
  }
  return block_sum(sum, red);
}

__device__ __forceinline__ void put_re(double* p, double v) { *p = v; }
__device__ __forceinline__ void put_re(cx<double>* p, double v) { *p = cx<double>{v, 0.0}; }

// End of the SpMV kernels: the sketch bins (summed over the waves; bins_all
// holds kWaves wave-major rows of s bins), ||x||^2 (when sketching), the
// window products and ||w||^2 into the tile's partial slots.  The values are
// summed per wave first, then one barrier (which also completes the bins)
// and a fixed-order sum over the waves: the same operations in the same
// order as one block_sum per value, with one barrier instead of three each.
template <class A, int NW = kWaves, int NT = kBlock>  // NW waves, NT threads per block
__device__ __forceinline__ void store_step_partials(A* __restrict__ part, int nb, int tile, int s, int sb,
                                                    int tw, const A* bins_all, double nx,
                                                    const A (&d)[kMaxWindow], double nw,
                                                    A (*wsum)[kMaxWindow + 2]) {
  constexpr int NV = kMaxWindow + 2;
  {
    A v[NV];
    v[0] = zero<A>();
    put_re(&v[0], s > 0 ? wave_sum(nx) : 0.0);
#pragma unroll
    for (int q = 0; q < kMaxWindow; ++q) v[1 + q] = q < tw ? wave_sum(d[q]) : zero<A>();
    v[NV - 1] = zero<A>();
    put_re(&v[NV - 1], wave_sum(nw));
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int i = 0; i < NV; ++i) wsum[threadIdx.x >> 6][i] = v[i];
  }
  __syncthreads();
  // (sb = 0: the sketch rows are another kernel's)
  for (int row = threadIdx.x; row < sb; row += NT) {
    A sum = bins_all[row];
    for (int q = 1; q < NW; ++q) sum += bins_all[q * sb + row];
    part[(int64_t)row * nb + tile] = sum;
  }
  // thread i < tw + 2 writes value i: ||x||^2 (when sketching) at row s, the
  // window products at s + 1 + q, ||w||^2 at s + 1 + tw (without the sketch
  // the rows start at 0 with the products)
  const int i = threadIdx.x;
  if (i >= (s > 0 ? 0 : 1) && i < tw + 2) {
    const int src = i <= tw ? i : NV - 1;
    A sum = wsum[0][src];
    for (int q = 1; q < NW; ++q) sum += wsum[q][src];
    part[(int64_t)(s > 0 ? s + i : i - 1) * nb + tile] = sum;
  }
}

// Row tile of a block in the streaming kernels.  Workgroups are dispatched
// to the 8 XCDs round robin, each XCD with its own L2: tile t of nb goes to
// the block that lands on XCD t / ceil-share, so an XCD works on a contiguous
// range of tiles.  An SpMV's halo rows then sit in the same L2, and the
// update kernel, tiled the same way, finds the vectors the SpMV just wrote
// there.  A bijection of [0, nb) for any nb.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, r = nb % kXcd;
  const int x = b % kXcd, k = b / kXcd;
  return x * q + (x < r ? x : r) + k;
}

// --------------------------------- SpMV + window products + input sketch --
// Each wave works on its own chunks of 64 rows, with no block barrier inside
// the row loop: a chunk whose entries fit the wave's staging buffer is read
// coalesced (lane e forms val[e] * x[ci[e]] into LDS, then lane r sums its row
// there); a longer chunk is read row by row.  The input vector x = p_{j-1} is
// read once more, coalesced, for its sketch and norm, and serves as the
// newest window vector.  (A grid-wide "last block" reduction would need a
// device-scope fence per block, which writes back the L2 of the block's XCD:
// the update kernel reduces the few scalars it needs instead.)
template <class T>
__global__ __launch_bounds__(kBlock) void k_spmv_sketch(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ val,
    const T* __restrict__ x, T* __restrict__ w, Window<T> win, int tw, SketchSpec sk, int wave_cap,
    int do_spmv, typename traits<T>::acc* __restrict__ part, int nb, const Ctrl* __restrict__ ctrl) {
  using A = typename traits<T>::acc;
  if (ctrl->halt) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = sk.s;  // 0: no sketch
  const int sb = sk.ext ? 0 : s;  // sketch bins of this kernel
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  A* bins = reinterpret_cast<A*>(smem_raw) + wv * sb;                   // this wave's sketch [sb]
  A* prod = reinterpret_cast<A*>(smem_raw) + kWaves * sb + wv * wave_cap;  // this wave's staging
  for (int i = lane; i < sb; i += 64) bins[i] = zero<A>();
  A d[kMaxWindow];
#pragma unroll
  for (int q = 0; q < kMaxWindow; ++q) d[q] = zero<A>();
  double nw = 0.0, nx = 0.0;
  const int tile = xcd_tile(blockIdx.x, nb);  // partial sums are stored by tile
  const int r0 = tile * kRowsSpmv;
  const int r1 = min(n, r0 + kRowsSpmv);
  for (int t0 = r0 + 64 * wv; t0 < r1; t0 += kBlock) {
    const int t1 = min(r1, t0 + 64);
    const int r = t0 + lane;
    const bool in = r < t1;
    // loads that do not depend on the row's entries go first
    A xa = zero<A>();
    A pw[kMaxWindow];
    int ra = 0, rb = 0;
    if (in) {
      xa = widen(x[r]);
      if (do_spmv) {
        ra = rp[r];
        rb = rp[r + 1];
#pragma unroll
        for (int q = 0; q < kMaxWindow; ++q)
          pw[q] = (q < tw && !(q + 1 == tw && win.p[q] == x)) ? widen(win.p[q][r]) : xa;
      }
    }
    A acc = zero<A>();
    if (do_spmv) {
      const int e0 = rp[t0], e1 = rp[t1];  // the same in every lane of the wave
      if (e1 - e0 <= wave_cap) {
        // all of the chunk's entries in flight at once, then their x gathers
        int cc[kWaveTileNnz / 64];
        A vv[kWaveTileNnz / 64];
#pragma unroll
        for (int u = 0; u < kWaveTileNnz / 64; ++u) {
          const int e = e0 + lane + 64 * u;
          if (e < e1) {
            cc[u] = ci[e];
            vv[u] = widen(val[e]);
          }
        }
#pragma unroll
        for (int u = 0; u < kWaveTileNnz / 64; ++u) {
          const int e = e0 + lane + 64 * u;
          if (e < e1) vv[u] = vv[u] * widen(x[cc[u]]);
        }
#pragma unroll
        for (int u = 0; u < kWaveTileNnz / 64; ++u) {
          const int e = e0 + lane + 64 * u;
          if (e < e1) prod[e - e0] = vv[u];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (in)
          for (int e = ra - e0; e < rb - e0; ++e) acc += prod[e];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else if (in) {
        for (int e = ra; e < rb; ++e) acc += widen(val[e]) * widen(x[ci[e]]);
      }
    }
    if (in) {
      if (s > 0) {
        const A xs = sk.src ? widen(static_cast<const T*>(sk.src)[r]) : xa;
        nx += abs2(xs);
        if (sb > 0) sketch_scatter(bins, r, xs, sk);
      }
      if (do_spmv) {
        const T wt = narrow<T>(acc);
        w[r] = wt;
        const A wa = widen(wt);
        nw += abs2(wa);
#pragma unroll
        for (int q = 0; q < kMaxWindow; ++q)
          if (q < tw) d[q] += conj(pw[q]) * wa;
      }
    }
  }
  __shared__ A wsum[kWaves][kMaxWindow + 2];
  store_step_partials(part, nb, tile, s, sb, tw, reinterpret_cast<const A*>(smem_raw), nx, d, nw, wsum);
}

template <class T>
static int spmv_wave_cap(int s) {
  using A = typename traits<T>::acc;
  const int budget = ((int)(kSpmvLds / sizeof(A)) - kWaves * s) / kWaves;
  // the staging loop is unrolled for kWaveTileNnz entries: the cap is that or nothing
  return budget < kWaveTileNnz ? 0 : kWaveTileNnz;
}

template <class T>
void launch_spmv_sketch(hipStream_t st, int n, const int* rp, const int* ci, const T* val, const T* x,
                        T* w, Window<T> win, int tw, SketchSpec sk, bool spmv,
                        typename traits<T>::acc* part, int nb, const Ctrl* ctrl, hipEvent_t e0,
                        hipEvent_t e1) {
  using A = typename traits<T>::acc;
  const int sb = sk.ext ? 0 : sk.s;
  const int cap = spmv ? spmv_wave_cap<T>(sb) : 0;
  const size_t lds = ((size_t)kWaves * sb + (size_t)kWaves * cap) * sizeof(A);
  const int dsp = spmv ? 1 : 0;
  if (e0)  // events recorded by the dispatch itself: the kernel's own duration
    hipExtLaunchKernelGGL(k_spmv_sketch<T>, dim3(nb), dim3(kBlock), lds, st, e0, e1, 0, n, rp, ci, val,
                          x, w, win, tw, sk, cap, dsp, part, nb, ctrl);
  else
    hipLaunchKernelGGL(k_spmv_sketch<T>, dim3(nb), dim3(kBlock), lds, st, n, rp, ci, val, x, w, win,
                       tw, sk, cap, dsp, part, nb, ctrl);
}

// ------------------------------ diagonal-storage SpMV + products + sketch --
// Thread per row over kRowsSpmv rows per block.  Every load is coalesced (the
// value streams, x shifted by each offset, the window vectors) and none sits
// behind a branch: column indices are clamped into [0, n) and the terms that
// fall outside the matrix are dropped by a select, so all loads of a row are
// in flight together before the sketch's LDS atomics and the arithmetic.
// ND > 0 fixes the number of diagonals at compile time (the common stencils);
// ND == 0 reads it from M.  TWM bounds the window length (2, or kMaxWindow for
// longer windows), so a short window's accumulators take no registers.  NT
// threads per block (512: 8 waves, 3 rows each over a 1536-row tile; 256 when
// 8 waves of sketch bins do not fit the LDS budget).
template <class T, int ND, int TWM, int NT, bool CM = false>
__global__ __launch_bounds__(NT) void k_spmv_dia_sketch(
    int n, DiaView<T> M, const T* __restrict__ x, T* __restrict__ w, Window<T> win, int tw, SketchSpec sk,
    int do_spmv, typename traits<T>::acc* __restrict__ part, int nb, const Ctrl* __restrict__ ctrl) {
  using A = typename traits<T>::acc;
  constexpr int KD = ND > 0 ? ND : kMaxDiag;
  // The halt flag is tested once the first row's loads are out, so its
  // latency overlaps theirs (a halted launch still reads one row per thread).
  const int halted = ctrl->halt;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = sk.s;  // 0: no sketch
  const int sb = sk.ext ? 0 : s;  // sketch bins of this kernel
  A* bins = reinterpret_cast<A*>(smem_raw) + (threadIdx.x >> 6) * sb;
  for (int i = threadIdx.x & 63; i < sb; i += 64) bins[i] = zero<A>();
  A d[kMaxWindow];
#pragma unroll
  for (int q = 0; q < kMaxWindow; ++q) d[q] = zero<A>();
  double nw = 0.0, nx = 0.0;
  const int tile = xcd_tile(blockIdx.x, nb);  // partial sums are stored by tile
  const int r0 = tile * kRowsSpmv;
  const int r1 = min(n, r0 + kRowsSpmv);
  if (!do_spmv) {
    for (int r = r0 + (int)threadIdx.x; r < r1; r += NT) {
      const A xa = widen(x[r]);
      if (halted) return;
      nx += abs2(xa);
      if (sb > 0) sketch_scatter(bins, r, xa, sk);
    }
  } else {
    const int nd = ND > 0 ? ND : M.ndiag;
    // In an Arnoldi step the newest window vector is x itself: its value is
    // already in a register.
    const int tl = (tw > 0 && win.p[tw - 1] == x) ? tw - 1 : tw;
    for (int r = r0 + (int)threadIdx.x; r < r1; r += NT) {
      const T xt = x[r];
      T vv[KD], xc[KD], pw[TWM];
#pragma unroll
      for (int q = 0; q < TWM; ++q)
        if (q < tl) pw[q] = win.p[q][r];
#pragma unroll
      for (int k = 0; k < KD; ++k) {
        if (ND > 0 || k < nd) {
          // (CM: a constant diagonal's value from the kernel argument, its
          // stream not read; the condition is the same for the whole grid)
          if (CM && ((M.cmask >> k) & 1u))
            vv[k] = M.cval[k];
          else
            vv[k] = M.val[(int64_t)k * n + r];
          xc[k] = x[min(max(r + M.off[k], 0), n - 1)];
        }
      }
      if (halted) return;
      const A xa = widen(xt);
      if (s > 0) {
        const A xs = sk.src ? widen(static_cast<const T*>(sk.src)[r]) : xa;
        nx += abs2(xs);
        if (sb > 0) sketch_scatter(bins, r, xs, sk);
      }
      A acc = zero<A>();
#pragma unroll
      for (int k = 0; k < KD; ++k) {
        if (ND > 0 || k < nd) {
          const int c = r + M.off[k];
          const A t = widen(vv[k]) * widen(xc[k]);
          acc += (c >= 0 && c < n) ? t : zero<A>();
        }
      }
      const T wt = narrow<T>(acc);
      w[r] = wt;
      const A wa = widen(wt);
      nw += abs2(wa);
#pragma unroll
      for (int q = 0; q < TWM; ++q)
        if (q < tw) d[q] += conj(q < tl ? widen(pw[q]) : xa) * wa;
    }
  }
  if (halted) return;
  __shared__ A wsum[NT / 64][kMaxWindow + 2];
  store_step_partials<A, NT / 64, NT>(part, nb, tile, s, sb, tw, reinterpret_cast<const A*>(smem_raw), nx, d,
                                      nw, wsum);
}

template <class T>
void launch_spmv_dia_sketch(hipStream_t st, int n, DiaView<T> M, const T* x, T* w, Window<T> win, int tw,
                            SketchSpec sk, bool spmv, typename traits<T>::acc* part, int nb,
                            const Ctrl* ctrl, hipEvent_t e0, hipEvent_t e1) {
  using A = typename traits<T>::acc;
  // 8 waves per block when their sketch bins fit the LDS budget, else 4 (the
  // generic instantiation); sdr_create keeps 4 waves' bins within it
  const int sb = sk.ext ? 0 : sk.s;
  const bool wide =
      (size_t)(kSpmvThreads / 64) * (sb + kMaxWindow + 2) * sizeof(A) <= (size_t)kSpmvLds;  // bins + wsum
  const int nt = wide ? kSpmvThreads : kBlock;
  const size_t lds = (size_t)(nt / 64) * sb * sizeof(A);
  const int dsp = spmv ? 1 : 0;
  void (*kern)(int, DiaView<T>, const T*, T*, Window<T>, int, SketchSpec, int, A*, int, const Ctrl*);
  if (wide && M.cmask != 0 && tw <= 3 && (M.ndiag == 5 || M.ndiag == 7)) {
    // constant diagonals (the stencils of constant-coefficient operators)
    if (tw <= 2)
      kern = M.ndiag == 5 ? k_spmv_dia_sketch<T, 5, 2, kSpmvThreads, true>
                          : k_spmv_dia_sketch<T, 7, 2, kSpmvThreads, true>;
    else
      kern = M.ndiag == 5 ? k_spmv_dia_sketch<T, 5, 3, kSpmvThreads, true>
                          : k_spmv_dia_sketch<T, 7, 3, kSpmvThreads, true>;
  } else if (!wide) {
    kern = k_spmv_dia_sketch<T, 0, kMaxWindow, kBlock>;
  } else if (tw <= 2) {
    switch (M.ndiag) {
      case 3: kern = k_spmv_dia_sketch<T, 3, 2, kSpmvThreads>; break;
      case 5: kern = k_spmv_dia_sketch<T, 5, 2, kSpmvThreads>; break;
      case 7: kern = k_spmv_dia_sketch<T, 7, 2, kSpmvThreads>; break;
      case 9: kern = k_spmv_dia_sketch<T, 9, 2, kSpmvThreads>; break;
      default: kern = k_spmv_dia_sketch<T, 0, 2, kSpmvThreads>; break;
    }
  } else if (tw <= 3) {
    switch (M.ndiag) {
      case 3: kern = k_spmv_dia_sketch<T, 3, 3, kSpmvThreads>; break;
      case 5: kern = k_spmv_dia_sketch<T, 5, 3, kSpmvThreads>; break;
      case 7: kern = k_spmv_dia_sketch<T, 7, 3, kSpmvThreads>; break;
      case 9: kern = k_spmv_dia_sketch<T, 9, 3, kSpmvThreads>; break;
      default: kern = k_spmv_dia_sketch<T, 0, 3, kSpmvThreads>; break;
    }
  } else {
    switch (M.ndiag) {
      case 3: kern = k_spmv_dia_sketch<T, 3, kMaxWindow, kSpmvThreads>; break;
      case 5: kern = k_spmv_dia_sketch<T, 5, kMaxWindow, kSpmvThreads>; break;
      case 7: kern = k_spmv_dia_sketch<T, 7, kMaxWindow, kSpmvThreads>; break;
      case 9: kern = k_spmv_dia_sketch<T, 9, kMaxWindow, kSpmvThreads>; break;
      default: kern = k_spmv_dia_sketch<T, 0, kMaxWindow, kSpmvThreads>; break;
    }
  }
  if (e0)
    hipExtLaunchKernelGGL(kern, dim3(nb), dim3(nt), lds, st, e0, e1, 0, n, M, x, w, win, tw, sk, dsp,
                          part, nb, ctrl);
  else
    hipLaunchKernelGGL(kern, dim3(nb), dim3(nt), lds, st, n, M, x, w, win, tw, sk, dsp, part, nb, ctrl);
}

template <class T>
__global__ void k_pack_dia(int64_t nnz, const typename traits<T>::acc* __restrict__ src,
                           const int* __restrict__ map, T* __restrict__ dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    dst[map[e]] = narrow<T>(src[e]);
}

template <class T>
void launch_pack_dia(hipStream_t st, int64_t nnz, const typename traits<T>::acc* src, const int* map, T* dst) {
  const int nb = (int)std::min<int64_t>((nnz + kBlock - 1) / kBlock, 65536);
  hipLaunchKernelGGL(k_pack_dia<T>, dim3(nb > 0 ? nb : 1), dim3(kBlock), 0, st, nnz, src, map, dst);
}

// One block per diagonal: every entry inside the matrix (rows with
// 0 <= r + off < n) compared bitwise with the first; the diagonal is constant
// when none differs.  A diagonal with no entry inside the matrix is not.
template <class T>
__global__ __launch_bounds__(kBlock) void k_dia_const(int n, DiaView<T> M, int* __restrict__ flags,
                                                      T* __restrict__ vals) {
  static_assert(sizeof(T) % sizeof(unsigned) == 0, "T");
  constexpr int NW = (int)(sizeof(T) / sizeof(unsigned));
  __shared__ int bad;
  const int d = blockIdx.x;
  const int off = M.off[d];
  const int ra = off < 0 ? -off : 0, rb = off > 0 ? n - off : n;
  if (threadIdx.x == 0) bad = ra < rb ? 0 : 1;
  __syncthreads();
  if (ra < rb) {
    const T* v = M.val + (int64_t)d * n;
    const T ref = v[ra];
    unsigned rw[NW];
    __builtin_memcpy(rw, &ref, sizeof(T));
    int mine = 0;
    for (int r = ra + (int)threadIdx.x; r < rb; r += kBlock) {
      const T e = v[r];
      unsigned ew[NW];
      __builtin_memcpy(ew, &e, sizeof(T));
#pragma unroll
      for (int q = 0; q < NW; ++q) mine |= ew[q] != rw[q];
    }
    if (mine) bad = 1;  // (every writer stores 1)
    __syncthreads();
    if (threadIdx.x == 0) {
      flags[d] = bad ? 0 : 1;
      vals[d] = ref;
    }
  } else if (threadIdx.x == 0) {
    flags[d] = 0;
    vals[d] = T{};
  }
}

template <class T>
void launch_dia_const(hipStream_t st, int n, DiaView<T> M, int* flags, T* vals) {
  hipLaunchKernelGGL(k_dia_const<T>, dim3(M.ndiag), dim3(kBlock), 0, st, n, M, flags, vals);
}

// ------------------------------------------- truncated orthogonalisation ---
// Prologue: nu_{j-1} = ||p_{j-1}|| and the window products from the SpMV
// partials of this step (columns s, s+1 .. s+tw), in the order every reducer
// uses.  Then p_j = (w - sum c_q p_q) / nu_{j-1} in place with
// c_q = <p_q, w> / nu_q^2: a pure stream over w and the window vectors, each
// thread with kUpdateRows independent rows in flight.
// NT threads per block (a multiple of kBlock): the first kBlock threads form
// the sums exactly as a kBlock-thread block would, so the bits do not depend
// on NT; a larger block repeats that reduction for fewer blocks.
template <class T, int TWM, int UR, int NT>  // TWM: bound on the window length tw; UR rows per thread
__global__ __launch_bounds__(NT) void k_update(
    int n, T* __restrict__ w, Window<T> win, int tw, const typename traits<T>::acc* __restrict__ part,
    int nb1, int s, double* __restrict__ nu, int i0, int jprev, const Ctrl* __restrict__ ctrl) {
  using A = typename traits<T>::acc;
  static_assert(NT % kBlock == 0, "NT");
  constexpr int NC = TWM + 1;
  const int halted = ctrl->halt;  // tested once the loads below are out
  __shared__ A red[NC * kWaves];
  const bool reducer = threadIdx.x < kBlock;  // (whole waves)
  // This step's partial sums (columns s .. s + tw, L2-resident) are loaded
  // first: their values return ahead of the stream loads issued after them,
  // so the block's reduction runs while the stream is still in flight.
  const A* pp = part + (int64_t)s * nb1;
  const int nc = tw + 1;
  A pv0[kPartRounds][NC];  // columns past nc re-read column nc - 1 and are not added
  if (reducer) {
#pragma unroll
    for (int u = 0; u < kPartRounds; ++u) {
      const int i = min((int)threadIdx.x + u * kBlock, nb1 - 1);
#pragma unroll
      for (int c = 0; c < NC; ++c) pv0[u][c] = pp[(int64_t)min(c, nc - 1) * nb1 + i];
    }
  }
  const int base = xcd_tile(blockIdx.x, gridDim.x) * (NT * UR) + (int)threadIdx.x;
  T wv[UR], pv[UR][TWM];
#pragma unroll
  for (int u = 0; u < UR; ++u) {
    const int r = min(base + u * NT, n - 1);
    wv[u] = w[r];
#pragma unroll
    for (int q = 0; q < TWM; ++q)
      if (q < tw) pv[u][q] = win.p[q][r];
  }
  double nqv[TWM];
#pragma unroll
  for (int q = 0; q < TWM; ++q) nqv[q] = (q < tw && i0 + q != jprev) ? nu[i0 + q] : 1.0;
  if (halted) return;
  // column sums in the order of col_sum: each reducer thread adds partials
  // threadIdx.x, + kBlock, + 2 kBlock, ... in increasing order, then the
  // waves in order (the grouping of the loads into rounds does not change it)
  A sums[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) sums[c] = zero<A>();
  if (reducer) {
#pragma unroll
    for (int u = 0; u < kPartRounds; ++u)
      if ((int)threadIdx.x + u * kBlock < nb1)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c < nc) sums[c] += pv0[u][c];
    for (int j0 = (int)threadIdx.x + kPartRounds * kBlock; j0 < nb1; j0 += 4 * kBlock) {
      A v[4][NC];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = min(j0 + u * kBlock, nb1 - 1);
#pragma unroll
        for (int c = 0; c < NC; ++c) v[u][c] = pp[(int64_t)min(c, nc - 1) * nb1 + i];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j0 + u * kBlock < nb1)
#pragma unroll
          for (int c = 0; c < NC; ++c)
            if (c < nc) sums[c] += v[u][c];
    }
  }
  {
    const int lane = threadIdx.x & 63, wv_ = threadIdx.x >> 6;
    if (reducer) {
#pragma unroll
      for (int c = 0; c < NC; ++c) sums[c] = wave_sum(sums[c]);
      if (lane == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) red[c * kWaves + wv_] = sums[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      A t = red[c * kWaves];
      for (int i = 1; i < kWaves; ++i) t += red[c * kWaves + i];
      sums[c] = t;
    }
  }
  const double nprev = sqrt(re(sums[0]));
  if (blockIdx.x == 0 && threadIdx.x == 0) nu[jprev] = nprev;
  A c[TWM];
#pragma unroll
  for (int q = 0; q < TWM; ++q) {
    if (q < tw) {
      const double nq = i0 + q == jprev ? nprev : nqv[q];
      c[q] = scale(sums[1 + q], 1.0 / (nq * nq));
    } else {
      c[q] = zero<A>();
    }
  }
  const double inv = 1.0 / nprev;
#pragma unroll
  for (int u = 0; u < UR; ++u) {
    const int r = base + u * NT;
    if (r < n) {
      A v = widen(wv[u]);
#pragma unroll
      for (int q = 0; q < TWM; ++q)
        if (q < tw) v -= c[q] * widen(pv[u][q]);
      w[r] = narrow<T>(scale(v, inv));
    }
  }
}

template <class T>
void launch_update(hipStream_t st, int n, T* w, Window<T> win, int tw,
                   const typename traits<T>::acc* part, int nb1, int s, double* nu, int i0, int jprev,
                   const Ctrl* ctrl, hipEvent_t e0, hipEvent_t e1) {
  // the window bound as a template parameter: a short window's rows take no
  // registers (t = 3, the complex workload's, is the common longer one).
  // Complex data take kUpdateThreads threads per block (half the blocks
  // repeat the reduction of the step's partials: 14.98-15.16 us against
  // 15.84 us per complex128 update at 1024^2); real data keep kBlock, where
  // the larger block was slower (6.7-6.8 against 6.2-6.6 us); the longest
  // window keeps kBlock too (its complex rows would spill at two waves per
  // SIMD)
  constexpr int NT = traits<T>::cpx ? kUpdateThreads : kBlock;
  const int nt = tw <= 3 ? NT : kBlock;
  const int nb = (n + nt * kUpdateRows - 1) / (nt * kUpdateRows);
  void (*kern)(int, T*, Window<T>, int, const typename traits<T>::acc*, int, int, double*, int, int,
               const Ctrl*) = tw <= 1   ? k_update<T, 1, kUpdateRows, NT>
                              : tw <= 2 ? k_update<T, 2, kUpdateRows, NT>
                              : tw <= 3 ? k_update<T, 3, kUpdateRows, NT>
                                        : k_update<T, kMaxWindow, kUpdateRows, kBlock>;
  if (e0)
    hipExtLaunchKernelGGL(kern, dim3(nb), dim3(nt), 0, st, e0, e1, 0, n, w, win, tw, part, nb1, s, nu,
                          i0, jprev, ctrl);
  else
    hipLaunchKernelGGL(kern, dim3(nb), dim3(nt), 0, st, n, w, win, tw, part, nb1, s, nu, i0, jprev,
                       ctrl);
}

// ------------------------------------------------ fixed-order reduction ---
template <class A>
__global__ __launch_bounds__(kBlock) void k_reduce_cols(const A* __restrict__ part, int nb,
                                                        int nscaled, double scl, A* __restrict__ out,
                                                        const Ctrl* __restrict__ ctrl, A* mirror) {
  if (ctrl && ctrl->halt) return;
  __shared__ A red[kWaves];
  const int col = blockIdx.x;
  const A sum = col_sum(part, nb, col, red);
  if (threadIdx.x == 0) {
    const A v = col < nscaled ? scale(sum, scl) : sum;
    out[col] = v;
    if (mirror) mirror[col] = v;
  }
}

template <class A>
void launch_reduce_cols(hipStream_t st, const A* part, int nb, int ncols, int nscaled,
                        double scl, A* out, const Ctrl* ctrl, A* mirror) {
  hipLaunchKernelGGL(k_reduce_cols<A>, dim3(ncols), dim3(kBlock), 0, st, part, nb, nscaled, scl, out,
                     ctrl, mirror);
}

// out[c] for c < ca from partA (c < nscaled scaled by scl), then cb columns of partB.
template <class A>
__global__ __launch_bounds__(kBlock) void k_reduce2(const A* __restrict__ pa, int nba, int ca,
                                                    int nscaled, double scl, const A* __restrict__ pb,
                                                    int nbb, A* __restrict__ out,
                                                    const Ctrl* __restrict__ ctrl) {
  if (ctrl->halt) return;
  __shared__ A red[kWaves];
  const int col = blockIdx.x;
  const A sum = col < ca ? col_sum(pa, nba, col, red) : col_sum(pb, nbb, col - ca, red);
  if (threadIdx.x == 0) out[col] = col < nscaled ? scale(sum, scl) : sum;
}

template <class A>
void launch_reduce2(hipStream_t st, const A* pa, int nba, int ca, int nscaled, double scl,
                    const A* pb, int nbb, int cb, A* out, const Ctrl* ctrl) {
  hipLaunchKernelGGL(k_reduce2<A>, dim3(ca + cb), dim3(kBlock), 0, st, pa, nba, ca, nscaled, scl, pb,
                     nbb, out, ctrl);
}

// col_sum of one column by a single wave: lane l stands in for the threads
// l, l + 64, l + 128 and l + 192 of a kBlock-thread block, each accumulating
// its partials in col_sum's order; the four wave sums are then added in wave
// order, as block_sum adds them.  The same bits as col_sum, with no LDS and
// no barrier.
template <class A>
__device__ __forceinline__ A col_sum_wave(const A* __restrict__ part, int nb, int col) {
  static_assert(kBlock == 4 * 64, "four waves per block");
  const int lane = threadIdx.x & 63;
  const A* p = part + (int64_t)col * nb;
  A acc[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) acc[w] = zero<A>();
  for (int i0 = lane; i0 < nb; i0 += 4 * kBlock) {
    A v[4][4];
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int u = 0; u < 4; ++u) v[w][u] = p[min(i0 + 64 * w + u * kBlock, nb - 1)];
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + 64 * w + u * kBlock < nb) acc[w] += v[w][u];
  }
  A sum = wave_sum(acc[0]);
#pragma unroll
  for (int w = 1; w < 4; ++w) sum += wave_sum(acc[w]);
  return sum;
}

// Reduced inputs of the least squares of steps j0 .. j0 + gridDim.y - 1, each
// into its slot of redb: [S p_j (s, scaled), ||p_j||^2] from the SpMV
// partials of step j+1, then the window products and ||w||^2 of step j.
// One wave per (column, step), four columns per block, each sum in the fixed
// order of col_sum (the order the update kernel uses for the same values).
template <class A>
__global__ __launch_bounds__(kBlock) void k_reduce_steps(const A* __restrict__ part1, int64_t slot1,
                                                         int nb1, int s, int j0, int t, int nslot,
                                                         double scl, A* __restrict__ redb,
                                                         int64_t slotr, const Ctrl* __restrict__ ctrl) {
  if (ctrl->halt) return;
  const int j = j0 + (int)blockIdx.y;
  const int tw = j - (j - t > 0 ? j - t : 0);
  const int col = (int)blockIdx.x * kWaves + ((int)threadIdx.x >> 6);
  if (col >= s + 1 + tw + 1) return;  // (whole waves)
  const A* pa = part1 + slot1 * ((j + 1) % nslot);
  const A* pb = part1 + slot1 * (j % nslot) + (int64_t)(s + 1) * nb1;
  const A sum = col < s + 1 ? col_sum_wave(pa, nb1, col) : col_sum_wave(pb, nb1, col - (s + 1));
  if ((threadIdx.x & 63) == 0) redb[slotr * (j % nslot) + col] = col < s ? scale(sum, scl) : sum;
}

template <class A>
void launch_reduce_steps(hipStream_t st, const A* part1, int64_t slot1, int nb1, int s, int j0, int j1,
                         int t, int nslot, double scl, A* redb, int64_t slotr, const Ctrl* ctrl) {
  const int ncol = s + 1 + kMaxWindow + 1;
  hipLaunchKernelGGL(k_reduce_steps<A>, dim3((ncol + kWaves - 1) / kWaves, j1 - j0 + 1), dim3(kBlock), 0, st,
                     part1, slot1, nb1, s, j0, t, nslot, scl, redb, slotr, ctrl);
}

// Cycle start: nu_0 = ||p_0|| and SV(:, 0) = S p_0 / nu_0 from a reduced sketch [s values, norm^2].
template <class A>
__global__ void k_init_v0(const A* __restrict__ red, int s, A* __restrict__ svcol, double* __restrict__ nu) {
  const double n0 = sqrt(re(red[s]));
  const double inv = n0 > 0.0 ? 1.0 / n0 : 0.0;
  for (int r = threadIdx.x; r < s; r += blockDim.x) svcol[r] = scale(red[r], inv);
  if (threadIdx.x == 0) nu[0] = n0;
}

template <class A>
void launch_init_v0(hipStream_t st, const A* red, int s, A* svcol, double* nu) {
  hipLaunchKernelGGL(k_init_v0<A>, dim3(1), dim3(kBlock), 0, st, red, s, svcol, nu);
}

// ------------------------------------------------ sketched least squares ---
// Step record (plain stores; the host reads them after synchronising) and,
// for the step that halts, the halt record published behind a system-scope
// fence: one fence per halt, none per step.
template <class A>
__device__ __forceinline__ void put_record(const LsqState<A>& S, int j, double sres, double nu, int flags,
                                           bool halt) {
  StepRec* rc = S.rec + j;
  rc->sres = sres;
  rc->nu = nu;
  rc->j = j;
  rc->flags = flags;
  if (halt) {
    HaltRec* h = S.halt;
    h->sres = sres;
    h->j = j;
    h->flags = flags;
    __threadfence_system();
    __hip_atomic_store(&h->seq, j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Residual control of one step (one thread): the safety-factor rule of
// Section 3.4 (sres < tol / safety), or the Givens estimate of Sections 4.5
// and 5: the step's sine is sres / sres_prev (the sketched residual falls by
// the Givens sine), the estimate grows by sqrt((s^2 + 2 eps (1 + c)) /
// (1 - eps^2)), and the check is due once it is below tol.
__device__ __forceinline__ bool control_due(Ctrl* c, double sres) {
  if (c->mode == 0) return sres < c->thresh;
  const double sp = c->sprev;
  double sn = sp > 0.0 ? sres / sp : 0.0;
  sn = sn < 1.0 ? sn : 1.0;
  const double cs = sqrt(fmax(0.0, 1.0 - sn * sn));
  const double e = c->eps;
  const double est = c->est * sqrt((sn * sn + 2.0 * e * (1.0 + cs)) / (1.0 - e * e));
  c->est = est;
  c->sprev = sres;
  return est < c->thresh;
}

// Cycle start of the control (one thread): sres0 is the sketched residual
// over span(U) alone (||S r0|| without a recycled block).
template <class A>
__device__ __forceinline__ void control_start(const LsqState<A>& S, int khat, double sres0, GivensInit gv) {
  Ctrl* c = S.ctrl;
  c->mode = gv.mode;
  if (gv.mode != 0) {
    c->eps = gv.eps;
    c->sprev = sres0;
    c->est = khat == 0 ? gv.beta : sres0 / sqrt(1.0 - gv.eps);
  }
  S.rec[0].sres = sres0;
}

// ||rho|| over the block (red: blockDim.x / 64 doubles), valid in every thread.
template <class A>
__device__ double rho_norm(const A* rho, int s, double* red) {
  double q = 0.0;
  for (int r = threadIdx.x; r < s; r += blockDim.x) q += abs2(rho[r]);
  return sqrt(block_sum(q, red));
}

constexpr int kLsqPrefetch = 16;  // staged elements per thread and chunk

// LDS layout of the least-squares kernels: a (s), acc (s), c (2 Lmax), then
// the staged chunk of Q (ch x s).  ch follows from the LDS budget.
template <class A>
__host__ __device__ inline int lsq_chunk(int s, int lmax) {
  const int budget = 60 * 1024 / (int)sizeof(A) - 2 * s - 2 * lmax;
  int ch = budget / s;
  const int cap = kLsqPrefetch * kLsqBlock / s;
  if (ch > cap) ch = cap;
  return ch < 1 ? 1 : ch;
}

// Append column a (in LDS, length s) to the QR factorisation Q R of SAW by
// classical Gram-Schmidt with one reorthogonalisation (Section 3.3 allows
// Householder or Gram-Schmidt with reorthogonalisation), then update the
// projected residual rho and z = Q^H S r0.  Each Gram-Schmidt pass reads Q
// once, chunk by chunk through LDS: the chunk's products with the pass input
// and its contribution to the update use the same staged data, and the next
// chunk's loads are issued before the current chunk is used.  Returns the
// sketched residual.
template <class A>
__device__ double qr_append(LsqState<A>& S, A* a, A* acc, A* cbuf, A* qs, int ch, A* red, int col,
                            int s, double rank_rtol, bool* rank_loss) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  const A* __restrict__ Q = S.Q;  // ld = s: columns are contiguous
  double n0 = 0.0;
  for (int r = tid; r < s; r += blockDim.x) n0 += abs2(a[r]);
  n0 = sqrt(block_sum(n0, (double*)red));
  for (int i = tid; i < col; i += blockDim.x) cbuf[i] = zero<A>();
  const int nch = (col + ch - 1) / ch;
  for (int pass = 0; pass < 2; ++pass) {
    for (int r = tid; r < s; r += blockDim.x) acc[r] = a[r];
    A pre[kLsqPrefetch];
    if (nch > 0) {
      const int tot = min(ch, col) * s;
#pragma unroll
      for (int u = 0; u < kLsqPrefetch; ++u) {
        const int idx = tid + u * kLsqBlock;
        pre[u] = idx < tot ? Q[idx] : zero<A>();
      }
    }
    for (int q = 0; q < nch; ++q) {
      const int c0 = q * ch, cw = min(ch, col - c0), tot = cw * s;
      __syncthreads();  // previous chunk fully consumed
#pragma unroll
      for (int u = 0; u < kLsqPrefetch; ++u) {
        const int idx = tid + u * kLsqBlock;
        if (idx < tot) qs[idx] = pre[u];
      }
      if (q + 1 < nch) {
        const int c1 = c0 + ch, tot1 = min(ch, col - c1) * s;
        const A* __restrict__ Qn = Q + (int64_t)c1 * s;
#pragma unroll
        for (int u = 0; u < kLsqPrefetch; ++u) {
          const int idx = tid + u * kLsqBlock;
          pre[u] = idx < tot1 ? Qn[idx] : zero<A>();
        }
      }
      __syncthreads();
      for (int i = wv; i < cw; i += nwv) {
        A d = zero<A>();
        for (int r = lane; r < s; r += 64) d += conj(qs[i * s + r]) * a[r];
        d = wave_sum(d);
        if (lane == 0) cbuf[col + c0 + i] = d;  // pass result in the upper half
      }
      __syncthreads();
      for (int r = tid; r < s; r += blockDim.x) {
        A v = acc[r];
        for (int i = 0; i < cw; ++i) v -= qs[i * s + r] * cbuf[col + c0 + i];
        acc[r] = v;
      }
    }
    __syncthreads();
    for (int r = tid; r < s; r += blockDim.x) a[r] = acc[r];
    for (int i = tid; i < col; i += blockDim.x) cbuf[i] += cbuf[col + i];
    __syncthreads();
  }
  double na = 0.0;
  for (int r = tid; r < s; r += blockDim.x) na += abs2(a[r]);
  na = sqrt(block_sum(na, (double*)red));
  const bool loss = !(na > rank_rtol * n0);
  *rank_loss = loss;
  const double inv = na > 0.0 ? 1.0 / na : 0.0;
  A* qc = S.Q + (int64_t)col * S.ldq;
  for (int r = tid; r < s; r += blockDim.x) {
    const A v = scale(a[r], inv);
    qc[r] = v;
    a[r] = v;  // keep the new q in LDS for the residual update
  }
  for (int i = tid; i < col; i += blockDim.x) S.R[(int64_t)col * S.ldr + i] = cbuf[i];
  if (tid == 0) {
    A d = zero<A>();
    *(double*)&d = na;
    S.R[(int64_t)col * S.ldr + col] = d;
  }
  __syncthreads();
  double sres;
  if (!loss) {
    A zc = zero<A>();
    for (int r = tid; r < s; r += blockDim.x) zc += conj(a[r]) * S.rho[r];
    zc = block_sum(zc, red);
    double rr = 0.0;
    for (int r = tid; r < s; r += blockDim.x) {
      const A v = S.rho[r] - a[r] * zc;
      S.rho[r] = v;
      rr += abs2(v);
    }
    sres = sqrt(block_sum(rr, (double*)red));
    if (tid == 0) S.z[col] = zc;
  } else {
    double rr = 0.0;
    for (int r = tid; r < s; r += blockDim.x) rr += abs2(S.rho[r]);
    sres = sqrt(block_sum(rr, (double*)red));
    if (tid == 0) S.z[col] = zero<A>();
  }
  __syncthreads();
  return sres;
}

// ---- register-resident variant ------------------------------------------
// Q (s x col, ld = s) is held in registers: lane l of wave w keeps rows
// l + 64 rr (rr < RL) of columns w + 8 cc (cc < CW), so one burst of
// coalesced loads brings the whole factor in.  Products with a column are a
// per-lane sum plus a wave reduction (every lane ends with the value); the
// update a - Q c is a per-lane sum reduced over the eight waves through LDS.
// Every wave keeps a full copy of the working vector (its rows per lane).
constexpr int kRegWaves = kLsqBlock / 64;

template <class A, int RL, int CW>
struct RegQ {
  A q[RL][CW];
};

template <class A, int RL, int CW>
__device__ __forceinline__ void regq_load(RegQ<A, RL, CW>& Q, const A* __restrict__ g, int s, int col) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int cc = 0; cc < CW; ++cc) {
    const int i = wv + kRegWaves * cc;
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      const int r = lane + 64 * rr;
      Q.q[rr][cc] = (i < col && r < s) ? g[(int64_t)i * s + r] : zero<A>();
    }
  }
}

// a (registers, rows lane + 64 rr) is orthogonalised against the col columns
// in Q (twice); returns ||a|| after and writes the R column (c1 + c2) for
// i < col into R, and the new unit column into Q's registers and into g.
template <class A, int RL, int CW>
__device__ double regq_append(RegQ<A, RL, CW>& Q, A (&a)[RL], A* __restrict__ g, A* __restrict__ Rcol,
                              A* lds_red /* kRegWaves * 64 * RL */, double* scr /* per wave */, int s,
                              int col, double rank_rtol, bool* loss) {
  constexpr int NC = CW * ncomp<A>::v;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double n0 = 0.0;
#pragma unroll
  for (int rr = 0; rr < RL; ++rr) n0 += abs2(a[rr]);
  n0 = sqrt(wave_sum(n0));
  // this wave holds columns wv + kRegWaves * cc; those at or beyond col are
  // zero (a wave with none skips the reduction; per-column branches would
  // break the interleaving of the reductions and cost more than they save)
  const int nact = col > wv ? (col - wv + kRegWaves - 1) / kRegWaves : 0;
  A ctot[CW];
#pragma unroll
  for (int cc = 0; cc < CW; ++cc) ctot[cc] = zero<A>();
  for (int pass = 0; pass < 2; ++pass) {
    double dd[NC];
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) {
      A d = zero<A>();
#pragma unroll
        for (int rr = 0; rr < RL; ++rr) d += conj(Q.q[rr][cc]) * a[rr];
      split_re(d, dd + cc * ncomp<A>::v);
    }
    if (nact > 0) wave_sums<NC>(dd, scr);
    A c[CW];
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) {
      join_re(c[cc], dd + cc * ncomp<A>::v);
      ctot[cc] += c[cc];
    }
    // partial update over this wave's columns, reduced over the waves
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      A u = zero<A>();
#pragma unroll
      for (int cc = 0; cc < CW; ++cc)
        u += Q.q[rr][cc] * c[cc];
      lds_red[(wv * RL + rr) * 64 + lane] = u;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      A u = lds_red[(0 * RL + rr) * 64 + lane];
      for (int w = 1; w < kRegWaves; ++w) u += lds_red[(w * RL + rr) * 64 + lane];
      a[rr] -= u;
    }
    __syncthreads();
  }
  // R column: entries of this wave's columns (lane 0 writes)
  if (lane == 0) {
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) {
      const int i = wv + kRegWaves * cc;
      if (i < col) Rcol[i] = ctot[cc];
    }
  }
  double na = 0.0;
#pragma unroll
  for (int rr = 0; rr < RL; ++rr) na += abs2(a[rr]);
  na = sqrt(wave_sum(na));
  *loss = !(na > rank_rtol * n0);
  const double inv = na > 0.0 ? 1.0 / na : 0.0;
#pragma unroll
  for (int rr = 0; rr < RL; ++rr) a[rr] = scale(a[rr], inv);
  // the new column joins Q: global memory (wave 0) and the owner wave's registers
  if (wv == 0) {
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      const int r = lane + 64 * rr;
      if (r < s) g[(int64_t)col * s + r] = a[rr];
    }
  }
  if (wv == col % kRegWaves) {
    const int cc = col / kRegWaves;
#pragma unroll
    for (int k = 0; k < CW; ++k)
      if (k == cc)
#pragma unroll
        for (int rr = 0; rr < RL; ++rr) Q.q[rr][k] = (lane + 64 * rr < s) ? a[rr] : zero<A>();
  }
  return na;
}

// projected residual update with the new unit column q (registers of every
// wave); wave 0 owns rho.  Returns the sketched residual (all threads).
template <class A, int RL>
__device__ double regq_residual(const A (&q)[RL], A* __restrict__ rho, A* __restrict__ zc_out,
                                bool skip, int s, double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (wv == 0) {
    A rv[RL];
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      const int r = lane + 64 * rr;
      rv[rr] = r < s ? rho[r] : zero<A>();
    }
    A zc = zero<A>();
    if (!skip) {
#pragma unroll
      for (int rr = 0; rr < RL; ++rr) zc += conj(q[rr]) * rv[rr];
      zc = wave_sum(zc);
#pragma unroll
      for (int rr = 0; rr < RL; ++rr) {
        rv[rr] -= q[rr] * zc;
        const int r = lane + 64 * rr;
        if (r < s) rho[r] = rv[rr];
      }
    }
    double rr2 = 0.0;
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) rr2 += abs2(rv[rr]);
    rr2 = wave_sum(rr2);
    if (lane == 0) {
      *zc_out = zc;
      *sh = sqrt(rr2);
    }
  }
  __syncthreads();
  return *sh;
}

template <class A, int RL, int CW>
__global__ __launch_bounds__(kLsqBlock) void k_lsq_step_reg(LsqState<A> S, int j, int khat, int m,
                                                            int t, int s, const A* __restrict__ red,
                                                            double brtol, double rank_rtol) {
  if (S.ctrl->halt) return;
  __shared__ A lds_red[kRegWaves * 64 * RL];
  __shared__ double scr_all[kRegWaves * 16 * (CW * ncomp<A>::v + 1)];
  __shared__ A hcol[kMaxWindow + 1];
  __shared__ int sh_break;
  __shared__ double sh_res;
  const int tid = threadIdx.x, lane = tid & 63;
  const int i0 = j - t > 0 ? j - t : 0;
  const int tw = j - i0;
  const int col = khat + j - 1;
  RegQ<A, RL, CW> Q;
  regq_load(Q, S.Q, s, col);  // issued first: in flight during the small work below
  const A* dots = red + s + 1;
  const double nuj = sqrt(re(red[s]));
  if (tid == 0) {
    const double nuprev = S.nu[j - 1];
    const double nw = sqrt(re(dots[tw]));
    const bool brk = !(nuj > brtol * nw / nuprev);  // H(j,j-1) vs ||A v_{j-1}||
    sh_break = brk;
    S.nu[j] = nuj;  // same reduction order as the update kernel's prologue
    for (int q = 0; q < tw; ++q) {
      const A h = scale(dots[q], 1.0 / (S.nu[i0 + q] * nuprev));
      hcol[q] = h;
      S.H[(int64_t)(j - 1) * S.ldh + i0 + q] = h;
    }
    A hs = zero<A>();
    *(double*)&hs = brk ? 0.0 : nuj;
    hcol[tw] = hs;
    S.H[(int64_t)(j - 1) * S.ldh + j] = hs;
  }
  __syncthreads();
  const bool brk = sh_break;
  // SV(:, j) and SAV(:, j-1) = SV(:, window + j) H(:, j-1), rows of this lane
  A a[RL];
  A* svj = S.SB + (int64_t)(khat + j) * S.ldsb;
  A* sawc = S.SAW + (int64_t)(khat + j - 1) * S.ldsaw;
#pragma unroll
  for (int rr = 0; rr < RL; ++rr) {
    const int r = lane + 64 * rr;
    A sum = zero<A>();
    if (r < s) {
      const A v = brk ? zero<A>() : scale(red[r], 1.0 / nuj);
      for (int q = 0; q < tw; ++q) sum += S.SB[(int64_t)(khat + i0 + q) * S.ldsb + r] * hcol[q];
      sum += v * hcol[tw];
      if (tid < 64) {
        svj[r] = v;
        sawc[r] = sum;
      }
    }
    a[rr] = sum;
  }
  bool loss = false;
  const double na =
      regq_append<A, RL, CW>(Q, a, S.Q, S.R + (int64_t)col * S.ldr, lds_red,
                             scr_all + (tid >> 6) * 16 * (CW * ncomp<A>::v + 1), s, col, rank_rtol, &loss);
  if (tid == 0) {
    A d = zero<A>();
    *(double*)&d = na;
    S.R[(int64_t)col * S.ldr + col] = d;
  }
  const double sres = regq_residual<A, RL>(a, S.rho, S.z + col, loss, s, &sh_res);
  if (tid == 0) {
    int flags = 0;
    if (brk) flags |= 2;
    if (loss) flags |= 4;
    const bool due = control_due(S.ctrl, sres);  // (updates the estimate: always evaluated)
    const bool halt = due || j == m || brk || loss;
    if (halt) flags |= 1;
    S.sres_hist[j] = sres;
    if (halt) {
      S.ctrl->halt = 1;
      S.ctrl->halt_j = j;
      S.ctrl->flags = flags;
    }
    put_record(S, j, sres, nuj, flags, halt);
  }
}

// Steps j0 .. j1 of the least squares in one launch: Q stays in registers,
// the projected residual rho in wave 0's registers and the SV columns of the
// truncation window in an LDS ring, so a step costs its QR append and little
// else.  The same arithmetic as k_lsq_step_reg, step after step; the launch
// stops after a step that raises the halt flag.
template <class A, int RL, int CW>
__global__ __launch_bounds__(kLsqBlock) void k_lsq_steps_reg(LsqState<A> S, int j0, int j1, int khat,
                                                             int m, int t, int s,
                                                             const A* __restrict__ redb, int64_t slotr,
                                                             int nslot, double brtol, double rank_rtol) {
  if (S.ctrl->halt) return;
  constexpr int SP = 64 * RL;  // ring pitch (>= s)
  __shared__ A lds_red[kRegWaves * 64 * RL];
  __shared__ double scr_all[kRegWaves * 16 * (CW * ncomp<A>::v + 1)];
  __shared__ A ring[kMaxWindow * SP];  // SV(:, k) at slot k % kMaxWindow
  __shared__ A hcol[kMaxWindow + 1];
  __shared__ int sh_break, sh_halt;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  RegQ<A, RL, CW> Q;
  regq_load(Q, S.Q, s, khat + j0 - 1);
  {
    const int i0 = j0 - t > 0 ? j0 - t : 0;
    for (int k = i0; k < j0; ++k)
      for (int r = tid; r < s; r += blockDim.x)
        ring[(k % kMaxWindow) * SP + r] = S.SB[(int64_t)(khat + k) * S.ldsb + r];
  }
  A rho[RL];
#pragma unroll
  for (int rr = 0; rr < RL; ++rr) {
    const int r = lane + 64 * rr;
    rho[rr] = (wv == 0 && r < s) ? S.rho[r] : zero<A>();
  }
  double* scr = scr_all + wv * 16 * (CW * ncomp<A>::v + 1);
  __syncthreads();
  for (int j = j0; j <= j1; ++j) {
    const A* red = redb + slotr * (j % nslot);
    const int i0 = j - t > 0 ? j - t : 0;
    const int tw = j - i0;
    const int col = khat + j - 1;
    const A* dots = red + s + 1;
    const double nuj = sqrt(re(red[s]));
    if (tid == 0) {
      const double nuprev = S.nu[j - 1];
      const double nw = sqrt(re(dots[tw]));
      const bool brk = !(nuj > brtol * nw / nuprev);  // H(j,j-1) vs ||A v_{j-1}||
      sh_break = brk;
      S.nu[j] = nuj;
      for (int q = 0; q < tw; ++q) {
        const A h = scale(dots[q], 1.0 / (S.nu[i0 + q] * nuprev));
        hcol[q] = h;
        S.H[(int64_t)(j - 1) * S.ldh + i0 + q] = h;
      }
      A hs = zero<A>();
      *(double*)&hs = brk ? 0.0 : nuj;
      hcol[tw] = hs;
      S.H[(int64_t)(j - 1) * S.ldh + j] = hs;
    }
    __syncthreads();
    const bool brk = sh_break;
    A a[RL], v[RL];
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      const int r = lane + 64 * rr;
      A sum = zero<A>();
      v[rr] = zero<A>();
      if (r < s) {
        v[rr] = brk ? zero<A>() : scale(red[r], 1.0 / nuj);
        for (int q = 0; q < tw; ++q) sum += ring[((i0 + q) % kMaxWindow) * SP + r] * hcol[q];
        sum += v[rr] * hcol[tw];
        if (wv == 0) {
          S.SB[(int64_t)(khat + j) * S.ldsb + r] = v[rr];
          S.SAW[(int64_t)(khat + j - 1) * S.ldsaw + r] = sum;
        }
      }
      a[rr] = sum;
    }
    bool loss = false;
    const double na = regq_append<A, RL, CW>(Q, a, S.Q, S.R + (int64_t)col * S.ldr, lds_red, scr, s, col,
                                             rank_rtol, &loss);
    // the window ring takes SV(:, j) (slot of SV(:, j - kMaxWindow), no longer needed)
    if (wv == 0) {
#pragma unroll
      for (int rr = 0; rr < RL; ++rr) {
        const int r = lane + 64 * rr;
        if (r < s) ring[(j % kMaxWindow) * SP + r] = v[rr];
      }
    }
    if (wv == 0) {
      A zc = zero<A>();
      if (!loss) {
#pragma unroll
        for (int rr = 0; rr < RL; ++rr) zc += conj(a[rr]) * rho[rr];
        zc = wave_sum(zc);
#pragma unroll
        for (int rr = 0; rr < RL; ++rr) rho[rr] -= a[rr] * zc;
      }
      double rr2 = 0.0;
#pragma unroll
      for (int rr = 0; rr < RL; ++rr) rr2 += abs2(rho[rr]);
      const double sres = sqrt(wave_sum(rr2));
      if (lane == 0) {
        A d = zero<A>();
        *(double*)&d = na;
        S.R[(int64_t)col * S.ldr + col] = d;
        S.z[col] = zc;
        int flags = 0;
        if (brk) flags |= 2;
        if (loss) flags |= 4;
        const bool due = control_due(S.ctrl, sres);  // (updates the estimate: always evaluated)
    const bool halt = due || j == m || brk || loss;
        if (halt) flags |= 1;
        S.sres_hist[j] = sres;
        if (halt) {
          S.ctrl->halt = 1;
          S.ctrl->halt_j = j;
          S.ctrl->flags = flags;
        }
        sh_halt = halt;
        put_record(S, j, sres, nuj, flags, halt);
      }
    }
    __syncthreads();
    if (sh_halt) break;
  }
  if (wv == 0) {
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      const int r = lane + 64 * rr;
      if (r < s) S.rho[r] = rho[rr];
    }
  }
}

template <class A, int RL, int CW>
__global__ __launch_bounds__(kLsqBlock) void k_lsq_init_reg(LsqState<A> S, int khat, int s,
                                                            const A* __restrict__ Sr, double rank_rtol,
                                                            GivensInit gv) {
  __shared__ A lds_red[kRegWaves * 64 * RL];
  __shared__ double scr_all[kRegWaves * 16 * (CW * ncomp<A>::v + 1)];
  __shared__ double sh_res;
  const int lane = threadIdx.x & 63;
  RegQ<A, RL, CW> Q;
#pragma unroll
  for (int cc = 0; cc < CW; ++cc)
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) Q.q[rr][cc] = zero<A>();
  for (int r = threadIdx.x; r < s; r += blockDim.x) S.rho[r] = Sr[r];
  __syncthreads();
  double sres = 0.0;
  for (int c = 0; c < khat; ++c) {
    A a[RL];
#pragma unroll
    for (int rr = 0; rr < RL; ++rr) {
      const int r = lane + 64 * rr;
      a[rr] = r < s ? S.SAW[(int64_t)c * S.ldsaw + r] : zero<A>();
    }
    bool loss = false;
    const double na =
        regq_append<A, RL, CW>(Q, a, S.Q, S.R + (int64_t)c * S.ldr, lds_red,
                               scr_all + (threadIdx.x >> 6) * 16 * (CW * ncomp<A>::v + 1), s, c,
                               rank_rtol, &loss);
    if (threadIdx.x == 0) {
      A d = zero<A>();
      *(double*)&d = na;
      S.R[(int64_t)c * S.ldr + c] = d;
    }
    sres = regq_residual<A, RL>(a, S.rho, S.z + c, loss, s, &sh_res);
  }
  if (khat == 0) sres = rho_norm(S.rho, s, (double*)lds_red);
  if (threadIdx.x == 0) {
    S.sres_hist[0] = sres;
    control_start(S, khat, sres, gv);
  }
}

// register shapes: rows per lane RL and columns per wave CW
template <class A>
static bool lsq_reg_shape(int s, int lmax, int* rl, int* cw) {
  const int need_rl = (s + 63) / 64;
  const int need_cw = (lmax + kRegWaves - 1) / kRegWaves;
  if (sizeof(A) == 8) {
    if (need_rl <= 2 && need_cw <= 8) { *rl = 2; *cw = 8; return true; }
    if (need_rl <= 2 && need_cw <= 16) { *rl = 2; *cw = 16; return true; }
    if (need_rl <= 4 && need_cw <= 16) { *rl = 4; *cw = 16; return true; }
  } else {
    if (need_rl <= 2 && need_cw <= 8) { *rl = 2; *cw = 8; return true; }
    if (need_rl <= 4 && need_cw <= 8) { *rl = 4; *cw = 8; return true; }
  }
  return false;
}

template <class A>
__global__ __launch_bounds__(kLsqBlock) void k_lsq_step(LsqState<A> S, int j, int khat, int m,
                                                        int t, int s, const A* __restrict__ red,
                                                        double brtol, double rank_rtol) {
  // red: [0, s) S p_j (scaled), [s] ||p_j||^2, [s+1, s+1+tw) window products,
  //      [s+1+tw] ||A p_{j-1}||^2
  if (S.ctrl->halt) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lmax = khat + m + 1;
  const int ch = lsq_chunk<A>(s, lmax);
  A* a = reinterpret_cast<A*>(smem_raw);  // s
  A* accb = a + s;                        // s
  A* cbuf = accb + s;                     // 2 * Lmax
  A* qs = cbuf + 2 * lmax;                // ch * s
  __shared__ A red_s[kLsqBlock / 64];
  __shared__ A hcol[kMaxWindow + 1];
  __shared__ int sh_break;
  const int tid = threadIdx.x;
  const int i0 = j - t > 0 ? j - t : 0;  // first window vector (0-based)
  const int tw = j - i0;
  const A* dots = red + s + 1;
  const double nuj = sqrt(re(red[s]));
  if (tid == 0) {
    const double nuprev = S.nu[j - 1];
    const double nw = sqrt(re(dots[tw]));
    const bool brk = !(nuj > brtol * nw / nuprev);  // H(j,j-1) vs ||A v_{j-1}||
    sh_break = brk;
    // same reduction order as the update kernel's prologue: identical bits
    S.nu[j] = nuj;
    for (int q = 0; q < tw; ++q) {
      const A h = scale(dots[q], 1.0 / (S.nu[i0 + q] * nuprev));
      hcol[q] = h;
      S.H[(int64_t)(j - 1) * S.ldh + i0 + q] = h;
    }
    A hs = zero<A>();
    *(double*)&hs = brk ? 0.0 : nuj;
    hcol[tw] = hs;
    S.H[(int64_t)(j - 1) * S.ldh + j] = hs;
  }
  __syncthreads();
  const bool brk = sh_break;
  A* svj = S.SB + (int64_t)(khat + j) * S.ldsb;
  for (int r = tid; r < s; r += blockDim.x) {
    const A v = brk ? zero<A>() : scale(red[r], 1.0 / nuj);
    svj[r] = v;
    A sum = zero<A>();
    for (int q = 0; q < tw; ++q) sum += S.SB[(int64_t)(khat + i0 + q) * S.ldsb + r] * hcol[q];
    sum += v * hcol[tw];
    a[r] = sum;
    S.SAW[(int64_t)(khat + j - 1) * S.ldsaw + r] = sum;
  }
  __syncthreads();
  bool loss = false;
  const double sres = qr_append(S, a, accb, cbuf, qs, ch, red_s, khat + j - 1, s, rank_rtol, &loss);
  if (tid == 0) {
    int flags = 0;
    if (brk) flags |= 2;
    if (loss) flags |= 4;
    const bool due = control_due(S.ctrl, sres);  // (updates the estimate: always evaluated)
    const bool halt = due || j == m || brk || loss;
    if (halt) flags |= 1;
    S.sres_hist[j] = sres;
    if (halt) {
      S.ctrl->halt = 1;
      S.ctrl->halt_j = j;
      S.ctrl->flags = flags;
    }
    put_record(S, j, sres, nuj, flags, halt);
  }
}

// register shapes instantiated per type: (2,8), (2,16), (4,16), (4,8) for
// real data, (2,8), (4,8) for complex (wider ones spill)
#define SDR_LSQ_REG_CASE(RL, CW, KER, ...)                                                  \
  if constexpr (sizeof(A) == 8 || CW == 8) {                                                \
    if (rl == RL && cw == CW) {                                                             \
      hipLaunchKernelGGL((KER<A, RL, CW>), dim3(1), dim3(kLsqBlock), 0, st, __VA_ARGS__);   \
      return;                                                                               \
    }                                                                                       \
  }

template <class A>
void launch_lsq_step(hipStream_t st, LsqState<A> S, int j, int khat, int m, int t, int s,
                     const A* red, double brtol, double rank_rtol) {
  int rl = 0, cw = 0;
  if (lsq_reg_shape<A>(s, khat + m + 1, &rl, &cw)) {
    SDR_LSQ_REG_CASE(2, 8, k_lsq_step_reg, S, j, khat, m, t, s, red, brtol, rank_rtol)
    SDR_LSQ_REG_CASE(2, 16, k_lsq_step_reg, S, j, khat, m, t, s, red, brtol, rank_rtol)
    SDR_LSQ_REG_CASE(4, 16, k_lsq_step_reg, S, j, khat, m, t, s, red, brtol, rank_rtol)
    SDR_LSQ_REG_CASE(4, 8, k_lsq_step_reg, S, j, khat, m, t, s, red, brtol, rank_rtol)
  }
  const int lmax = khat + m + 1;
  const size_t lds = (size_t)(2 * s + 2 * lmax + lsq_chunk<A>(s, lmax) * s) * sizeof(A);
  hipLaunchKernelGGL(k_lsq_step<A>, dim3(1), dim3(kLsqBlock), lds, st, S, j, khat, m, t, s, red,
                     brtol, rank_rtol);
}

// ---- block variant --------------------------------------------------------
// For shapes whose factor does not fit the registers (a wide sketch, complex
// data), the steps of a launch are taken in blocks of up to kBlkCols columns
// by block classical Gram-Schmidt with reorthogonalisation (BCGS2): the new
// SAV columns W are projected against the committed factor Q, the remainder
// is factorised inside the block by CGS2 (W1 = Q1 R1), Q1 is projected once
// more and factorised again (Q2 R2), so that
//   W = Q (P1 + P2 R1) + Q2 (R2 R1),
// which appends Q2 to Q and [P1 + P2 R1; R2 R1] to R.  Q is swept four times
// per block instead of four times per column, and each sweep is a product
// with up to eight columns at once.  The steps are then finished one by one
// in the order of the sequential kernels (projected residual, residual
// control, records), and only the steps up to the one that halts are
// committed: the columns of Q and R beyond it are rewritten before they are
// read if the cycle resumes.
constexpr int kBlkThreads = 1024;
constexpr int kBlkWaves = kBlkThreads / 64;
constexpr int kBlkCols = 8;     // columns per block (the product lanes are 8 row groups x 8 columns)
constexpr int kBlkMaxS = 4096;  // largest sketch taken by the block kernel

// LDS pitch of the block's columns: >= s and 2 mod 16, so that the rows read
// by one product instruction (eight consecutive rows of each of the eight
// columns) fall in different banks.
__host__ __device__ inline int blk_pitch(int s) { return ((s + 13) / 16) * 16 + 2; }

__device__ __forceinline__ double shfl_xor_v(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ cx<double> shfl_xor_v(cx<double> v, int m) {
  return {__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64)};
}

// P(i, b) = Q(:, i)^H X(:, b) for i < ncol, b < nb (P row major, stride
// kBlkCols; rows ncol .. up to the next multiple of 8 are set to zero).  A
// wave takes eight columns of Q at a time; lane (c, g) = (lane / 8, lane % 8)
// sums rows g, g + 8, ... of column c of the group against all block columns,
// so one load instruction reads eight consecutive rows (a 128-byte line) of
// each of eight columns.  The eight row groups are combined by DPP inside
// each half row (quad swaps, then the half-row mirror), a fixed order.
// Waves wv < nb first store ||X(:, wv)|| in n0 when n0 is given.
template <class A>
__device__ void blk_project(const A* __restrict__ Q, int ldq, int ncol, int s, const A* X, int ps, int nb,
                            A* P, double* n0) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (n0 != nullptr && wv < nb) {
    double q = 0.0;
    for (int r = lane; r < s; r += 64) q += abs2(X[wv * ps + r]);
    q = wave_sum(q);
    if (lane == 0) n0[wv] = sqrt(q);
  }
  const int c = lane >> 3, g = lane & 7;
  for (int i0 = 8 * wv; i0 < ncol; i0 += 8 * kBlkWaves) {
    const int i = i0 + c;
    const A* __restrict__ qc = Q + (int64_t)min(i, ncol - 1) * ldq;
    A acc[kBlkCols];
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) acc[b] = zero<A>();
#pragma unroll 4
    for (int r = g; r < s; r += 8) {
      const A q = conj(qc[r]);
#pragma unroll
      for (int b = 0; b < kBlkCols; ++b)
        if (b < nb) acc[b] += q * X[b * ps + r];
    }
    double d[kBlkCols * ncomp<A>::v];
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) split_re(acc[b], d + b * ncomp<A>::v);
#pragma unroll
    for (int e = 0; e < kBlkCols * ncomp<A>::v; ++e) {
      d[e] += dpp_mov<0xB1>(d[e]);
      d[e] += dpp_mov<0x4E>(d[e]);
      d[e] += dpp_mov<0x141>(d[e]);
    }
    if (g == 0) {
#pragma unroll
      for (int b = 0; b < kBlkCols; ++b) {
        A v;
        join_re(v, d + b * ncomp<A>::v);
        if (b < nb) P[i * kBlkCols + b] = i < ncol ? v : zero<A>();
      }
    }
  }
}

// X(:, b) -= Q(:, 0:ncol) P(0:ncol, b) for b < nb, one thread per row and
// half block; the row's columns stay in registers over the sweep, and the
// next eight Q entries are loaded while the current eight are applied (P's
// zero rows past ncol pad the last group, a multiple of U rows).
template <class A, int CB>
__device__ __forceinline__ void blk_update_rows(const A* __restrict__ Q, int ldq, int ncol, int r, int c0,
                                                A* X, int ps, int nb, const A* P) {
  constexpr int U = sizeof(A) == 16 ? 4 : 8;  // (register budget)
  A acc[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) acc[c] = c0 + c < nb ? X[(c0 + c) * ps + r] : zero<A>();
  A qn[U];
#pragma unroll
  for (int u = 0; u < U; ++u) qn[u] = ncol > 0 ? Q[(int64_t)min(u, ncol - 1) * ldq + r] : zero<A>();
  for (int i = 0; i < ncol; i += U) {
    A q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = qn[u];
    if (i + U < ncol) {
#pragma unroll
      for (int u = 0; u < U; ++u) qn[u] = Q[(int64_t)min(i + U + u, ncol - 1) * ldq + r];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[c] -= q[u] * P[(i + u) * kBlkCols + c0 + c];
  }
#pragma unroll
  for (int c = 0; c < CB; ++c)
    if (c0 + c < nb) X[(c0 + c) * ps + r] = acc[c];
}

template <class A>
__device__ void blk_update(const A* __restrict__ Q, int ldq, int ncol, int s, A* X, int ps, int nb,
                           const A* P) {
  constexpr int CB = kBlkCols / 2;
  for (int idx = threadIdx.x; idx < 2 * s; idx += kBlkThreads) {
    const int h = idx / s, r = idx - h * s;
    blk_update_rows<A, CB>(Q, ldq, ncol, r, h * CB, X, ps, nb, P);
  }
}

// CGS2 inside the block: X(:, 0:nb) = Xq Rm, Xq overwriting X, Rm upper
// triangular (column major, stride kBlkCols, real positive diagonal; zero
// below it).  A zero remainder gives a zero column and Rm(b, b) = 0.
template <class A>
__device__ void blk_qr(A* X, int ps, int s, int nb, A* Rm, A* dcur, A* dsum, double* sh_na) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = 0; b < nb; ++b) {
    A* xb = X + b * ps;
    for (int pass = 0; pass < 2 && b > 0; ++pass) {
      if (wv < b) {
        A d = zero<A>();
        for (int r = lane; r < s; r += 64) d += conj(X[wv * ps + r]) * xb[r];
        d = wave_sum(d);
        if (lane == 0) dcur[wv] = d;
      }
      __syncthreads();
      for (int r = tid; r < s; r += kBlkThreads) {
        A v = xb[r];
        for (int c = 0; c < b; ++c) v -= X[c * ps + r] * dcur[c];
        xb[r] = v;
      }
      if (tid == 0)
        for (int c = 0; c < b; ++c) dsum[c] = pass == 0 ? dcur[c] : dsum[c] + dcur[c];
      __syncthreads();
    }
    if (wv == 0) {
      double q = 0.0;
      for (int r = lane; r < s; r += 64) q += abs2(xb[r]);
      q = sqrt(wave_sum(q));
      if (lane == 0) *sh_na = q;
    }
    __syncthreads();
    const double na = *sh_na;
    const double inv = na > 0.0 ? 1.0 / na : 0.0;
    for (int r = tid; r < s; r += kBlkThreads) xb[r] = scale(xb[r], inv);
    if (tid < kBlkCols) {
      A v = zero<A>();
      if (tid < b) v = dsum[tid];
      if (tid == b) *(double*)&v = na;
      Rm[b * kBlkCols + tid] = v;
    }
    __syncthreads();
  }
}

template <class A>
__global__ __launch_bounds__(kBlkThreads) void k_lsq_block(LsqState<A> S, int j0, int j1, int khat, int m,
                                                           int t, int s, const A* __restrict__ redb,
                                                           int64_t slotr, int nslot, double brtol,
                                                           double rank_rtol, int bc, int prow) {
  if (S.ctrl->halt) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ps = blk_pitch(s);
  A* X = reinterpret_cast<A*>(smem_raw);  // ps x bc
  A* P = X + ps * bc;                      // prow x kBlkCols
  A* R1 = P + prow * kBlkCols;             // kBlkCols x kBlkCols, column major
  A* R2 = R1 + kBlkCols * kBlkCols;
  A* rhol = R2 + kBlkCols * kBlkCols;      // s: the projected residual (finishing wave)
  __shared__ A hc[kBlkCols][kMaxWindow + 1];
  __shared__ A RB[kBlkCols * kBlkCols];
  __shared__ A dcur[kBlkCols], dsum[kBlkCols];
  __shared__ double nujs[kBlkCols], n0[kBlkCols], sh_na;
  __shared__ int brks[kBlkCols], sh_halt, sh_last;
  __shared__ Ctrl cl;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int jb = j0; jb <= j1; jb += bc) {
    const int nb = min(bc, j1 - jb + 1);
    const int col0 = khat + jb - 1;  // committed columns of Q
    // H columns, breakdown tests and norms of the block's steps, one thread
    // per step (each norm is recomputed from its step's sums: the same bits)
    if (tid < nb) {
      const int b = tid, j = jb + b;
      const A* red = redb + slotr * (j % nslot);
      const int i0 = j - t > 0 ? j - t : 0, tw = j - i0;
      const A* dots = red + s + 1;
      const double nuj = sqrt(re(red[s]));
      const double nw = sqrt(re(dots[tw]));
      const double nuprev = b == 0 ? S.nu[jb - 1] : sqrt(re(redb[slotr * ((j - 1) % nslot) + s]));
      const bool brk = !(nuj > brtol * nw / nuprev);  // H(j,j-1) vs ||A v_{j-1}||
      for (int q = 0; q < tw; ++q) {
        const int i = i0 + q;
        const double nui = i < jb ? S.nu[i] : sqrt(re(redb[slotr * (i % nslot) + s]));
        hc[b][q] = scale(dots[q], 1.0 / (nui * nuprev));
      }
      A hs = zero<A>();
      *(double*)&hs = brk ? 0.0 : nuj;
      hc[b][tw] = hs;
      nujs[b] = nuj;
      brks[b] = brk;
    }
    __syncthreads();
    // SV and SAV columns (SAV(:, j) = SV(:, window) H(window, j)), one thread
    // per row: every load first (the block's sketch sums and the window
    // columns before the block), the SV values into X, then the SAV columns
    // in place, last first, so that column b still finds the SV values of
    // the columns before it.  The same sums in the same order as the
    // column-by-column kernels.
    for (int r = tid; r < s; r += kBlkThreads) {
      A wpre[kMaxWindow];
#pragma unroll
      for (int p = 0; p < kMaxWindow; ++p) {
        const int i = jb - kMaxWindow + p;
        wpre[p] = (i >= 0 && i >= jb - t) ? S.SB[(int64_t)(khat + i) * S.ldsb + r] : zero<A>();
      }
      A raw[kBlkCols];
#pragma unroll
      for (int b = 0; b < kBlkCols; ++b) raw[b] = b < nb ? redb[slotr * ((jb + b) % nslot) + r] : zero<A>();
#pragma unroll
      for (int b = 0; b < kBlkCols; ++b)
        if (b < nb) {
          const A v = brks[b] ? zero<A>() : scale(raw[b], 1.0 / nujs[b]);
          X[b * ps + r] = v;
          S.SB[(int64_t)(khat + jb + b) * S.ldsb + r] = v;
        }
#pragma unroll 1
      for (int b = nb - 1; b >= 0; --b) {
          const int j = jb + b, i0 = j - t > 0 ? j - t : 0, tw = j - i0;
          A sum = zero<A>();
          for (int q = 0; q < tw; ++q) {
            const int e = i0 + q - jb;  // window column relative to the block
            A w = e >= 0 ? X[max(e, 0) * ps + r] : zero<A>();
#pragma unroll
            for (int p = 0; p < kMaxWindow; ++p)
              if (e == p - kMaxWindow) w = wpre[p];
            sum += w * hc[b][q];
          }
          sum += X[b * ps + r] * hc[b][tw];
          X[b * ps + r] = sum;
          S.SAW[(int64_t)(khat + j - 1) * S.ldsaw + r] = sum;
        }
    }
    __syncthreads();
    // first projection: P1 = Q^H W (stored as the R entries above the block), W1 = W - Q P1
    blk_project(S.Q, S.ldq, col0, s, X, ps, nb, P, n0);
    __syncthreads();
    for (int i = tid; i < col0; i += kBlkThreads)
      for (int b = 0; b < nb; ++b) S.R[(int64_t)(col0 + b) * S.ldr + i] = P[i * kBlkCols + b];
    blk_update(S.Q, S.ldq, col0, s, X, ps, nb, P);
    __syncthreads();
    blk_qr(X, ps, s, nb, R1, dcur, dsum, &sh_na);  // W1 = Q1 R1
    // second projection: P2 = Q^H Q1, Q1 - Q P2 = Q2 R2; R above the block
    // becomes P1 + P2 R1 (each thread reads back what it stored)
    blk_project(S.Q, S.ldq, col0, s, X, ps, nb, P, (double*)nullptr);
    __syncthreads();
    for (int i = tid; i < col0; i += kBlkThreads)
      for (int b = 0; b < nb; ++b) {
        A u = zero<A>();
        for (int c = 0; c <= b; ++c) u += P[i * kBlkCols + c] * R1[b * kBlkCols + c];
        A* rp = S.R + (int64_t)(col0 + b) * S.ldr + i;
        *rp = *rp + u;
      }
    blk_update(S.Q, S.ldq, col0, s, X, ps, nb, P);
    __syncthreads();
    blk_qr(X, ps, s, nb, R2, dcur, dsum, &sh_na);
    // the block's R = R2 R1, then the steps in order (one wave)
    if (wv == 0) {
      const int c = lane >> 3, b = lane & 7;
      A v = zero<A>();
      if (c <= b && b < nb)
        for (int e = c; e <= b; ++e) v += R2[e * kBlkCols + c] * R1[b * kBlkCols + e];
      RB[b * kBlkCols + c] = v;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int r = lane; r < s; r += 64) rhol[r] = S.rho[r];
      if (lane == 0) cl = *S.ctrl;  // the control block, kept in LDS and written back
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      int last = nb - 1, halted = 0;
      for (int bb = 0; bb < nb; ++bb) {
        const int j = jb + bb, col = col0 + bb;
        const double na = re(RB[bb * kBlkCols + bb]);
        const bool loss = !(na > rank_rtol * n0[bb]);
        A zc = zero<A>();
        const A* qb = X + bb * ps;
        if (!loss) {
          for (int r = lane; r < s; r += 64) zc += conj(qb[r]) * rhol[r];
          zc = wave_sum(zc);
        }
        double rr2 = 0.0;
        for (int r = lane; r < s; r += 64) {
          A v = rhol[r];
          if (!loss) {
            v -= qb[r] * zc;
            rhol[r] = v;
          }
          rr2 += abs2(v);
        }
        const double sres = sqrt(wave_sum(rr2));
        int hv = 0;
        if (lane == 0) {
          const bool brk = brks[bb];
          const int i0 = j - t > 0 ? j - t : 0, tw = j - i0;
          S.nu[j] = nujs[bb];
          for (int q = 0; q <= tw; ++q) S.H[(int64_t)(j - 1) * S.ldh + i0 + q] = hc[bb][q];
          S.z[col] = zc;
          int flags = 0;
          if (brk) flags |= 2;
          if (loss) flags |= 4;
          const bool due = control_due(&cl, sres);  // (updates the estimate: always evaluated)
          const bool halt = due || j == m || brk || loss;
          if (halt) flags |= 1;
          S.sres_hist[j] = sres;
          if (halt) {
            S.ctrl->est = cl.est;
            S.ctrl->sprev = cl.sprev;
            S.ctrl->halt = 1;
            S.ctrl->halt_j = j;
            S.ctrl->flags = flags;
          }
          put_record(S, j, sres, nujs[bb], flags, halt);
          hv = halt;
        }
        hv = __shfl(hv, 0, 64);
        if (hv) {
          last = bb;
          halted = 1;
          break;
        }
      }
      for (int r = lane; r < s; r += 64) S.rho[r] = rhol[r];
      if (lane == 0 && !halted) {
        S.ctrl->est = cl.est;
        S.ctrl->sprev = cl.sprev;
      }
      if (lane == 0) {
        sh_last = last;
        sh_halt = halted;
      }
    }
    __syncthreads();
    // commit Q and the block's R up to the last finished step
    const int last = sh_last;
    for (int idx = tid; idx < (last + 1) * s; idx += kBlkThreads) {
      const int b = idx / s, r = idx - b * s;
      S.Q[(int64_t)(col0 + b) * S.ldq + r] = X[b * ps + r];
    }
    if (tid < kBlkCols * kBlkCols) {
      const int c = tid >> 3, b = tid & 7;
      if (c <= b && b <= last) S.R[(int64_t)(col0 + b) * S.ldr + col0 + c] = RB[b * kBlkCols + c];
    }
    if (sh_halt) return;
    __threadfence_block();
    __syncthreads();
  }
}

// Columns per block of the block kernel for this launch (0: it does not fit).
template <class A>
static int lsq_block_cols(int s, int prow, size_t* lds) {
  if (s > kBlkMaxS) return 0;
  static int limit[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (limit[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
    limit[dev] = std::min(v, 160 * 1024) - 4096;  // room for the kernel's static LDS
  }
  for (int bc = kBlkCols; bc >= 1; --bc) {
    const size_t bytes =
        ((size_t)blk_pitch(s) * bc + (size_t)prow * kBlkCols + 2 * kBlkCols * kBlkCols + s) * sizeof(A);
    if (bytes <= (size_t)limit[dev]) {
      *lds = bytes;
      return bc;
    }
  }
  return 0;
}

// ---- block variant on several workgroups ------------------------------------
// The same block Gram-Schmidt as k_lsq_block, split at its sweeps over Q so
// that each sweep runs on many workgroups: the step headers and the block W
// (k_mblk_head), the projection P = Q^H W (k_mblk_proj, a workgroup per eight
// columns of Q), the update W -= Q P (k_mblk_upd, a workgroup per 64 rows),
// the CGS2 inside the block (k_mblk_qr), the second projection and update,
// then the second in-block factorisation with the steps finished in order
// (k_mblk_fin).  The in-block kernels hold the block in registers: lane l of
// wave w keeps rows 64 (NW u + w) + l, u < RPL, of the eight columns (NW <= 4
// waves, s <= 64 NW RPL; rows past s hold zeros), so their sums are DPP
// steps and, with several waves, one LDS exchange.  Every kernel returns at
// once when the halt flag is set.  (The least squares of a cycle runs once
// the Arnoldi chain has drained, so the sweeps have the GPU to themselves.)
constexpr int kMblkMaxWaves = 4;   // waves of the in-block kernels
constexpr int kMblkHeadThreads = 1024;
constexpr int kMblkSweepThreads = 1024;
constexpr int kMblkSweepWaves = kMblkSweepThreads / 64;
// LDS of the in-block kernels' shared buffer: the Gram staging (waves x 36
// pairs x 2 parts x 8 groups) or the cross-wave sums (2 x kMblkSweepWaves x
// 32) with the per-wave wave_sums scratch (16 x 33), whichever is larger
constexpr int kMblkPool = (kMblkMaxWaves * 36 * 2 * 8 > 2 * kMblkSweepWaves * 32 + kMblkMaxWaves * 16 * 33)
                              ? kMblkMaxWaves * 36 * 2 * 8
                              : 2 * kMblkSweepWaves * 32 + kMblkMaxWaves * 16 * 33;

// Workgroup sums of NV per-lane values: every thread gets every sum, the same
// bits on every call.  Wave sums first; with nw > 1 waves the wave sums are
// added in wave order through xs (2 halves of kMblkSweepWaves x 32 doubles,
// used alternately, so one barrier per call keeps a later call from
// overwriting sums not yet read).  scr: this wave's wave_sums scratch.
template <int NV>
__device__ __forceinline__ void grp_sums(double (&d)[NV], double* scr, double* xs, int nw, int& ph) {
  if constexpr (NV == 8 || NV == 16 || NV == 32) {
    wave_sums<NV>(d, scr);
  } else {
#pragma unroll
    for (int c = 0; c < NV; ++c) d[c] = wave_sum(d[c]);
  }
  if (nw > 1) {
    double* x = xs + ph * (kMblkSweepWaves * 32);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane < NV) {
      double v = d[0];
#pragma unroll
      for (int c = 1; c < NV; ++c)
        if (lane == c) v = d[c];
      x[wv * 32 + lane] = v;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double t = x[c];
      for (int w = 1; w < nw; ++w) t += x[w * 32 + c];
      d[c] = t;
    }
    ph ^= 1;
  }
}

template <class A, int RPL>
__device__ __forceinline__ int mblk_row(int u, int nw) {
  return 64 * (nw * u + (int)(threadIdx.x >> 6)) + (int)(threadIdx.x & 63);
}

// acc + conj(a) b and acc - a b as chains of fused multiply-adds (four for
// complex data): the in-block kernels' inner products and updates, whose
// rounding need not match any other kernel's.
__device__ __forceinline__ double fmac_conj(double acc, double a, double b) { return fma(a, b, acc); }
__device__ __forceinline__ cx<double> fmac_conj(cx<double> acc, cx<double> a, cx<double> b) {
  return {fma(a.y, b.y, fma(a.x, b.x, acc.x)), fma(-a.y, b.x, fma(a.x, b.y, acc.y))};
}
__device__ __forceinline__ double fmsub(double acc, double a, double b) { return fma(-a, b, acc); }
__device__ __forceinline__ cx<double> fmsub(cx<double> acc, cx<double> a, cx<double> b) {
  return {fma(a.y, b.y, fma(-a.x, b.x, acc.x)), fma(-a.y, b.x, fma(-a.x, b.y, acc.y))};
}

// One projection pass of column B against the columns before it (NV packed
// sums: the projections first, the squared norm of column B last when
// with_norm): d = X(:, 0:B)^H X(:, B), X(:, B) -= X(:, 0:B) d.  Returns the
// squared norm (with_norm) and the projections' squared moduli in corr.
template <class A, int RPL, int B, int NV>
__device__ __forceinline__ double mblk_pass(A (&X)[kBlkCols][RPL], bool with_norm, A (&dsum)[kBlkCols], bool first,
                                            double* corr, double* scr, double* xs, int nw, int& ph) {
  constexpr int NC = ncomp<A>::v;
  static_assert(B * NC + 1 <= NV, "packing");
  double d[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) d[e] = 0.0;
#pragma unroll
  for (int c = 0; c < B; ++c) {
    A acc = zero<A>();
#pragma unroll
    for (int u = 0; u < RPL; ++u) acc = fmac_conj(acc, X[c][u], X[B][u]);
    split_re(acc, d + c * NC);
  }
  if (with_norm) {
#pragma unroll
    for (int u = 0; u < RPL; ++u) d[NV - 1] += abs2(X[B][u]);
  }
  grp_sums<NV>(d, scr, xs, nw, ph);
  A dc[B > 0 ? B : 1];
  double cr = 0.0;
#pragma unroll
  for (int c = 0; c < B; ++c) {
    join_re(dc[c], d + c * NC);
    cr += abs2(dc[c]);
  }
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    A v = X[B][u];
#pragma unroll
    for (int c = 0; c < B; ++c) v = fmsub(v, X[c][u], dc[c]);
    X[B][u] = v;
  }
#pragma unroll
  for (int c = 0; c < B; ++c) dsum[c] = first ? dc[c] : dsum[c] + dc[c];
  *corr = cr;
  return d[NV - 1];
}

// Column B of the in-block CGS2 (see mblk_qr).
template <class A, int RPL, int B>
__device__ __forceinline__ void mblk_qr_col(A (&X)[kBlkCols][RPL], int nb, A* Rm, double* scr, double* xs, int nw,
                                            int& ph) {
  if (B >= nb) return;
  constexpr int NC = ncomp<A>::v;
  constexpr int NV = B * NC + 1 <= 8 ? 8 : 16;  // the projections and the norm, packed
  A dsum[kBlkCols];
#pragma unroll
  for (int c = 0; c < kBlkCols; ++c) dsum[c] = zero<A>();
  double na2 = 0.0, corr = 0.0;
  bool explicit_norm = B == 0;
  if constexpr (B > 0) {
    mblk_pass<A, RPL, B, NV>(X, false, dsum, true, &corr, scr, xs, nw, ph);
    const double n2 = mblk_pass<A, RPL, B, NV>(X, true, dsum, false, &corr, scr, xs, nw, ph);
    na2 = n2 - corr;
    explicit_norm = !(corr <= 0.25 * n2);
  }
  if (explicit_norm) {
    double q[1] = {0.0};
#pragma unroll
    for (int u = 0; u < RPL; ++u) q[0] += abs2(X[B][u]);
    grp_sums<1>(q, scr, xs, nw, ph);
    na2 = q[0];
  }
  const double na = sqrt(fmax(na2, 0.0));
  const double inv = na > 0.0 ? 1.0 / na : 0.0;
#pragma unroll
  for (int u = 0; u < RPL; ++u) X[B][u] = scale(X[B][u], inv);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < kBlkCols; ++c) {
      A v = c < B ? dsum[c] : zero<A>();
      if (c == B) *(double*)&v = na;
      Rm[B * kBlkCols + c] = v;
    }
  }
}

// CGS2 of the register block: X(:, 0:nb) = Xq Rm, Xq overwriting X; Rm
// upper triangular (column major, stride kBlkCols, real non-negative
// diagonal, zeros below), written by thread 0.  Column b takes two workgroup
// sums: the projections on the columns before it, then the projections of the
// remainder together with its squared norm; the norm after the second
// (small) correction is that squared norm less the corrections' squares
// (Pythagoras), or a third sum when the correction is not small against the
// remainder (a column nearly in the span of those before it).  A zero
// remainder gives a zero column and Rm(b, b) = 0.
template <class A, int RPL>
__device__ void mblk_qr(A (&X)[kBlkCols][RPL], int nb, A* Rm, double* scr, double* xs, int nw, int& ph) {
  static_assert(kBlkCols == 8, "columns");
  static_assert((kBlkCols - 1) * ncomp<A>::v + 1 <= 16, "packing");
  mblk_qr_col<A, RPL, 0>(X, nb, Rm, scr, xs, nw, ph);
  mblk_qr_col<A, RPL, 1>(X, nb, Rm, scr, xs, nw, ph);
  mblk_qr_col<A, RPL, 2>(X, nb, Rm, scr, xs, nw, ph);
  mblk_qr_col<A, RPL, 3>(X, nb, Rm, scr, xs, nw, ph);
  mblk_qr_col<A, RPL, 4>(X, nb, Rm, scr, xs, nw, ph);
  mblk_qr_col<A, RPL, 5>(X, nb, Rm, scr, xs, nw, ph);
  mblk_qr_col<A, RPL, 6>(X, nb, Rm, scr, xs, nw, ph);
  mblk_qr_col<A, RPL, 7>(X, nb, Rm, scr, xs, nw, ph);
}

__device__ __forceinline__ double shfl_v(double v, int l) { return __shfl(v, l, 64); }
__device__ __forceinline__ cx<double> shfl_v(cx<double> v, int l) { return {__shfl(v.x, l, 64), __shfl(v.y, l, 64)}; }
__device__ __forceinline__ double read_lane_v(double v, int l) { return read_lane(v, l); }
__device__ __forceinline__ cx<double> read_lane_v(cx<double> v, int l) { return {read_lane(v.x, l), read_lane(v.y, l)}; }

// Cholesky QR of the register block, the in-block factorisation when the
// block is well conditioned: G = X^H X (each pair's lane sums added over
// groups of eight lanes by DPP, then through LDS, gbuf: nw x 36 x 2 x 8
// doubles, by lane (a, b) of each wave in a fixed order), G = Rm^H Rm, X <- X Rm^-1 row by
// row.  Inside block Gram-Schmidt with
// reorthogonalisation this is as stable as CGS2 while the block's condition
// number stays far below eps^(-1/2); a pivot below 1e-8 of its diagonal
// entry (a column within about 1e-4 of the span of those before it, a zero
// column) returns false with X untouched, and the caller takes CGS2.  The
// factorisation runs on the lanes of each wave alike: lane (a, b) = (lane /
// 8, lane % 8) holds G(a, b), row j of Rm is formed at step j and reaches
// the other lanes by shuffles; columns nb .. 7 get a unit pivot.
template <class A, int RPL>
__device__ bool mblk_cholqr(A (&X)[kBlkCols][RPL], int nb, A* Rm, double* gbuf) {
  static_assert(kBlkCols == 8, "one wave holds the 8 x 8 factor");
  constexpr int NC = ncomp<A>::v;
  constexpr int NP = kBlkCols * (kBlkCols + 1) / 2;  // pairs i <= j
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // each pair's lane sums, added over groups of eight lanes (DPP), into
  // gbuf[wave][pair][part][group]
  {
    int p = 0;
#pragma unroll
    for (int i = 0; i < kBlkCols; ++i)
#pragma unroll
      for (int j = i; j < kBlkCols; ++j, ++p) {
        A acc = zero<A>();
#pragma unroll
        for (int u = 0; u < RPL; ++u) acc = fmac_conj(acc, X[i][u], X[j][u]);
        double t[NC];
        split_re(acc, t);
#pragma unroll
        for (int h = 0; h < NC; ++h) {
          t[h] += dpp_mov<0xB1>(t[h]);
          t[h] += dpp_mov<0x4E>(t[h]);
          t[h] += dpp_mov<0x141>(t[h]);
          if ((lane & 7) == 0) gbuf[((wv * NP + p) * NC + h) * 8 + (lane >> 3)] = t[h];
        }
      }
  }
  __syncthreads();
  const int ra = lane >> 3, cb = lane & 7;
  A g = zero<A>();
  if (ra <= cb) {
    const int p = ra * kBlkCols - ra * (ra - 1) / 2 + (cb - ra);
    double t[NC];
#pragma unroll
    for (int h = 0; h < NC; ++h) t[h] = 0.0;
    for (int w = 0; w < nw; ++w)
#pragma unroll
      for (int h = 0; h < NC; ++h)
#pragma unroll
        for (int q = 0; q < 8; ++q) t[h] += gbuf[((w * NP + p) * NC + h) * 8 + q];
    join_re(g, t);
  }
  __syncthreads();  // (gbuf's buffer is the sums' scratch of what follows)
  if (ra >= nb || cb >= nb) {
    g = zero<A>();
    if (ra == cb) *(double*)&g = 1.0;
  }
  const double gdiag = re(g);
  bool ok = true;
  double inv[kBlkCols];
#pragma unroll
  for (int j = 0; j < kBlkCols; ++j) {
    const double d = read_lane(re(g), j * 9);  // the pivot, lane (j, j)
    ok = ok && (j >= nb || d > 1e-8 * read_lane(gdiag, j * 9));
    const double r = sqrt(fmax(d, 0.0));
    inv[j] = r > 0.0 ? 1.0 / r : 0.0;
    if (ra == j) {
      if (cb == j) {
        g = zero<A>();
        *(double*)&g = r;
      } else if (cb > j) {
        g = scale(g, inv[j]);
      }
    }
    const A rja = shfl_v(g, j * 8 + ra), rjb = shfl_v(g, j * 8 + cb);
    if (ra > j && ra <= cb) g = fmsub(g, conj(rja), rjb);
  }
  if (!ok) return false;
  // lane (c, b), c <= b, holds Rm(c, b); column j of Xq = (X(:, j) -
  // sum_{k<j} Xq(:, k) Rm(k, j)) / Rm(j, j), the earlier columns final first
#pragma unroll
  for (int j = 0; j < kBlkCols; ++j) {
    A rkj[kBlkCols];
#pragma unroll
    for (int k = 0; k < j; ++k) rkj[k] = read_lane_v(g, k * 8 + j);
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      A v = X[j][u];
#pragma unroll
      for (int k = 0; k < j; ++k) v = fmsub(v, X[k][u], rkj[k]);
      X[j][u] = scale(v, inv[j]);
    }
  }
  if (threadIdx.x < 64) Rm[cb * kBlkCols + ra] = (ra <= cb && cb < nb) ? g : zero<A>();
  return true;
}

// Step headers (a thread per step) and the block's SV and SAV columns into
// S.SB, S.SAW and bw.W (ld s), a thread per row; ||W(:, b)|| into bw.n0.
// The same sums in the same order as the column-by-column kernels.
template <class A>
__global__ __launch_bounds__(kMblkHeadThreads) void k_mblk_head(LsqState<A> S, int jb, int nb, int khat, int t,
                                                                int s, const A* __restrict__ redb, int64_t slotr,
                                                                int nslot, double brtol) {
  if (S.ctrl->halt) return;
  const BlkWork<A> B = S.bw;
  __shared__ A hc[kBlkCols][kMaxWindow + 1];
  __shared__ double nujs[kBlkCols];
  __shared__ int brks[kBlkCols], tws[kBlkCols];
  __shared__ double scr_all[(kMblkHeadThreads / 64) * 16 * (kBlkCols + 1)];
  __shared__ double xs[2 * kMblkSweepWaves * 32];
  const int tid = threadIdx.x, wv = tid >> 6, nw = blockDim.x >> 6;
  // the first row's loads are issued before the headers are formed
  A wpre[kMaxWindow], x[kBlkCols];
  auto load_row = [&](int r) {
#pragma unroll
    for (int p = 0; p < kMaxWindow; ++p) {
      const int i = jb - kMaxWindow + p;
      wpre[p] = (i >= 0 && i >= jb - t) ? S.SB[(int64_t)(khat + i) * S.ldsb + r] : zero<A>();
    }
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) x[b] = b < nb ? redb[slotr * ((jb + b) % nslot) + r] : zero<A>();
  };
  if (tid < s) load_row(tid);
  if (tid < nb) {
    const int b = tid, j = jb + b;
    const A* red = redb + slotr * (j % nslot);
    const int i0 = j - t > 0 ? j - t : 0, tw = j - i0;
    const A* dots = red + s + 1;
    const double nuj = sqrt(re(red[s]));
    const double nw2 = sqrt(re(dots[tw]));
    const double nuprev = b == 0 ? S.nu[jb - 1] : sqrt(re(redb[slotr * ((j - 1) % nslot) + s]));
    const bool brk = !(nuj > brtol * nw2 / nuprev);  // H(j,j-1) vs ||A v_{j-1}||
    for (int q = 0; q < tw; ++q) {
      const int i = i0 + q;
      const double nui = i < jb ? S.nu[i] : sqrt(re(redb[slotr * (i % nslot) + s]));
      hc[b][q] = scale(dots[q], 1.0 / (nui * nuprev));
    }
    A hs = zero<A>();
    *(double*)&hs = brk ? 0.0 : nuj;
    hc[b][tw] = hs;
    nujs[b] = nuj;
    brks[b] = brk;
    tws[b] = tw;
    for (int q = 0; q <= kMaxWindow; ++q) B.hc[b * (kMaxWindow + 1) + q] = q <= tw ? hc[b][q] : zero<A>();
    B.nuj[b] = nuj;
    B.brk[b] = brk;
  }
  __syncthreads();
  double nn[kBlkCols];
#pragma unroll
  for (int b = 0; b < kBlkCols; ++b) nn[b] = 0.0;
  for (int r = tid; r < s; r += blockDim.x) {
    if (r != tid) load_row(r);
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b)
      if (b < nb) {
        x[b] = brks[b] ? zero<A>() : scale(x[b], 1.0 / nujs[b]);
        S.SB[(int64_t)(khat + jb + b) * S.ldsb + r] = x[b];
      }
    // SAV(:, j) = SV(:, window) H(window, j), last column first so that
    // column b still finds the SV values before it; window column j - d sits
    // at block column b - d, or before the block (wpre) when that is < 0
#pragma unroll
    for (int b = kBlkCols - 1; b >= 0; --b)
      if (b < nb) {
        const int tw = tws[b];
        A sum = zero<A>();
#pragma unroll
        for (int d = kMaxWindow; d >= 1; --d)
          if (d <= tw) {
            const A w = b - d >= 0 ? x[b - d >= 0 ? b - d : 0] : wpre[kMaxWindow + b - d >= 0 ? kMaxWindow + b - d : 0];
            sum += w * hc[b][tw - d];
          }
        sum += x[b] * hc[b][tw];
        x[b] = sum;
        S.SAW[(int64_t)(khat + jb + b - 1) * S.ldsaw + r] = sum;
        B.W[b * s + r] = sum;
        nn[b] += abs2(sum);
      }
  }
  int ph = 0;
  grp_sums<kBlkCols>(nn, scr_all + wv * 16 * (kBlkCols + 1), xs, nw, ph);
  if (tid < kBlkCols) {
    double v = nn[0];
#pragma unroll
    for (int b = 1; b < kBlkCols; ++b)
      if (tid == b) v = nn[b];
    B.n0[tid] = sqrt(v);
  }
}

// The cycle's recycled columns, a block of nb from column c0: SAW's columns
// into bw.W (ld s), their norms into bw.n0; with c0 = 0 also rho = S r0.
template <class A>
__global__ __launch_bounds__(kMblkHeadThreads) void k_mblk_init_head(LsqState<A> S, int c0, int nb, int s,
                                                                     const A* __restrict__ Sr) {
  const BlkWork<A> B = S.bw;
  __shared__ double scr_all[(kMblkHeadThreads / 64) * 16 * (kBlkCols + 1)];
  __shared__ double xs[2 * kMblkSweepWaves * 32];
  const int tid = threadIdx.x, wv = tid >> 6, nw = blockDim.x >> 6;
  double nn[kBlkCols];
#pragma unroll
  for (int b = 0; b < kBlkCols; ++b) nn[b] = 0.0;
  for (int r = tid; r < s; r += blockDim.x) {
    if (c0 == 0) S.rho[r] = Sr[r];
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b)
      if (b < nb) {
        const A v = S.SAW[(int64_t)(c0 + b) * S.ldsaw + r];
        B.W[b * s + r] = v;
        nn[b] += abs2(v);
      }
  }
  int ph = 0;
  grp_sums<kBlkCols>(nn, scr_all + wv * 16 * (kBlkCols + 1), xs, nw, ph);
  if (tid < kBlkCols) {
    double v = nn[0];
#pragma unroll
    for (int b = 1; b < kBlkCols; ++b)
      if (tid == b) v = nn[b];
    B.n0[tid] = sqrt(v);
  }
}

// P(i, b) = Q(:, i)^H W(:, b) for i < ncol, b < nb (rows ncol .. the next
// multiple of 8 set to zero), and the R entries above the block, Rtop(i, b)
// = R(i, col0 + b): the first projection stores them (Rtop = P1), the second
// (with R1) adds P2 R1 to them (Rtop = P1 + P2 R1).  A workgroup per eight
// columns of Q; its waves take a share of the row groups each (lane (c, g):
// column c, rows g, g + 8, ...: one load instruction reads eight consecutive
// rows of each of eight columns), combined by DPP within a wave and through
// LDS across the waves in wave order.
template <class A>
__global__ __launch_bounds__(kMblkSweepThreads) void k_mblk_proj(const A* __restrict__ Q, int ldq, int ncol, int s,
                                                                 const A* __restrict__ W, int nb, A* __restrict__ P,
                                                                 A* __restrict__ Rtop, int ldr,
                                                                 const A* __restrict__ R1,
                                                                 const Ctrl* __restrict__ ctrl) {
  if (ctrl->halt) return;
  __shared__ A part[kMblkSweepWaves][kBlkCols][kBlkCols];
  __shared__ A pfin[kBlkCols][kBlkCols];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane >> 3, g = lane & 7;
  const int i0 = blockIdx.x * 8, i = i0 + c;
  const A* __restrict__ qc = Q + (int64_t)min(i, ncol - 1) * ldq;
  const int ngrp = (s + 7) / 8;  // rows g + 8 k, k < ngrp
  const int k0 = wv * ngrp / kMblkSweepWaves, k1 = (wv + 1) * ngrp / kMblkSweepWaves;
  A acc[kBlkCols];
#pragma unroll
  for (int b = 0; b < kBlkCols; ++b) acc[b] = zero<A>();
  for (int k = k0; k < k1; ++k) {
    const int r = min(g + 8 * k, s - 1);
    const A q = g + 8 * k < s ? conj(qc[r]) : zero<A>();
    A w[kBlkCols];
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) w[b] = b < nb ? W[b * s + r] : zero<A>();
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) acc[b] += q * w[b];
  }
  double d[kBlkCols * ncomp<A>::v];
#pragma unroll
  for (int b = 0; b < kBlkCols; ++b) split_re(acc[b], d + b * ncomp<A>::v);
#pragma unroll
  for (int e = 0; e < kBlkCols * ncomp<A>::v; ++e) {
    d[e] += dpp_mov<0xB1>(d[e]);
    d[e] += dpp_mov<0x4E>(d[e]);
    d[e] += dpp_mov<0x141>(d[e]);
  }
  if (g == 0) {
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) join_re(part[wv][c][b], d + b * ncomp<A>::v);
  }
  __syncthreads();
  const int cc = threadIdx.x >> 3, b = threadIdx.x & 7, ii = i0 + cc;
  A v = zero<A>();
  if (threadIdx.x < 64) {
    v = part[0][cc][b];
#pragma unroll
    for (int w = 1; w < kMblkSweepWaves; ++w) v += part[w][cc][b];
    if (b < nb) P[ii * kBlkCols + b] = ii < ncol ? v : zero<A>();
    if (R1 == nullptr && b < nb && ii < ncol) Rtop[(int64_t)b * ldr + ii] = v;
    pfin[cc][b] = v;
  }
  if (R1 == nullptr) return;
  __syncthreads();
  if (threadIdx.x < 64 && b < nb && ii < ncol) {
    A u = zero<A>();
    for (int c = 0; c <= b; ++c) u += pfin[cc][c] * R1[b * kBlkCols + c];
    A* rp = Rtop + (int64_t)b * ldr + ii;
    *rp = *rp + u;
  }
}

// W(r, b) -= sum_i Q(r, i) P(i, b): a workgroup per 64 rows, a lane per row;
// its waves take consecutive shares of the columns of Q (one load
// instruction reads 64 consecutive rows of a column; P's row is the same for
// the whole wave: scalar loads), and the partial sums of each entry are added
// in wave order through LDS (dynamic: kMblkSweepWaves x kBlkCols x 64).
template <class A>
__global__ __launch_bounds__(kMblkSweepThreads) void k_mblk_upd(const A* __restrict__ Q, int ldq, int ncol, int s,
                                                                A* __restrict__ W, int nb, const A* __restrict__ P,
                                                                const Ctrl* __restrict__ ctrl) {
  if (ctrl->halt) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  A* part = reinterpret_cast<A*>(smem_raw);
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = blockIdx.x * 64 + lane, rr = min(r, s - 1);
  const int c0 = wv * ncol / kMblkSweepWaves, c1 = (wv + 1) * ncol / kMblkSweepWaves;
  A acc[kBlkCols];
#pragma unroll
  for (int b = 0; b < kBlkCols; ++b) acc[b] = zero<A>();
  int i = c0;
  for (; i + 4 <= c1; i += 4) {
    A q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = Q[(int64_t)(i + u) * ldq + rr];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int b = 0; b < kBlkCols; ++b) acc[b] += q[u] * P[(i + u) * kBlkCols + b];
  }
  for (; i < c1; ++i) {
    const A q = Q[(int64_t)i * ldq + rr];
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) acc[b] += q * P[i * kBlkCols + b];
  }
#pragma unroll
  for (int b = 0; b < kBlkCols; ++b) part[(wv * kBlkCols + b) * 64 + lane] = acc[b];
  __syncthreads();
  // wave w < nb finishes block column w
  if (r < s && wv < nb) {
    A v = part[wv * 64 + lane];
    for (int w = 1; w < kMblkSweepWaves; ++w) v += part[(w * kBlkCols + wv) * 64 + lane];
    W[wv * s + r] -= v;
  }
}

// CGS2 inside the block: bw.W = Q1 R1 in place, R1 into bw.R1.
template <class A, int RPL>
__global__ __launch_bounds__(64 * kMblkMaxWaves) void k_mblk_qr(LsqState<A> S, int nb, int s) {
  if (S.ctrl->halt) return;
  // the Gram staging of the Cholesky QR and the sums' scratch of the CGS2
  // fallback share one buffer: they are never live together
  __shared__ double pool[kMblkPool];
  double* gbuf = pool;
  double* xs = pool;
  double* scr = pool + 2 * kMblkSweepWaves * 32 + (threadIdx.x >> 6) * 16 * 33;
  const int nw = blockDim.x >> 6;
  A X[kBlkCols][RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int r = mblk_row<A, RPL>(u, nw);
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) X[b][u] = (r < s && b < nb) ? S.bw.W[b * s + r] : zero<A>();
  }
  int ph = 0;
  if (!mblk_cholqr<A, RPL>(X, nb, S.bw.R1, gbuf)) mblk_qr<A, RPL>(X, nb, S.bw.R1, scr, xs, nw, ph);
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int r = mblk_row<A, RPL>(u, nw);
    if (r < s) {
#pragma unroll
      for (int b = 0; b < kBlkCols; ++b)
        if (b < nb) S.bw.W[b * s + r] = X[b][u];
    }
  }
}

// The second in-block factorisation (bw.W = Q2 R2), the block's R = R2 R1
// (the entries above it were completed by the second projection), then the
// steps in order (projected residual, residual control, records) and the
// commit of Q and R up to the last finished step.
template <class A, int RPL>
__global__ __launch_bounds__(64 * kMblkMaxWaves) void k_mblk_fin(LsqState<A> S, int jb, int nb, int m, int t,
                                                                 int s, int col0, double rank_rtol, int mode,
                                                                 GivensInit gv) {
  if (S.ctrl->halt) return;
  constexpr int NC = ncomp<A>::v;
  const BlkWork<A> B = S.bw;
  __shared__ double pool[kMblkPool];  // (the Gram staging, then the sums' scratch)
  double* gbuf = pool;
  double* xs = pool;
  __shared__ A R1[kBlkCols * kBlkCols], R2[kBlkCols * kBlkCols], RB[kBlkCols * kBlkCols];
  __shared__ A hcs[kBlkCols * (kMaxWindow + 1)];
  __shared__ double nujs[kBlkCols], n0s[kBlkCols];
  __shared__ int brks[kBlkCols];
  __shared__ int sh_halt;  // the last finished step of the block
  __shared__ Ctrl cl;
  const int tid = threadIdx.x, nw = blockDim.x >> 6, wv = tid >> 6;
  double* scr = pool + 2 * kMblkSweepWaves * 32 + wv * 16 * 33;
  if (tid < kBlkCols * (kMaxWindow + 1)) hcs[tid] = B.hc[tid];
  if (tid < kBlkCols) {
    nujs[tid] = B.nuj[tid];
    n0s[tid] = B.n0[tid];
    brks[tid] = B.brk[tid];
  }
  A X[kBlkCols][RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int r = mblk_row<A, RPL>(u, nw);
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) X[b][u] = (r < s && b < nb) ? B.W[b * s + r] : zero<A>();
  }
  A rh[RPL];  // the projected residual
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int r = mblk_row<A, RPL>(u, nw);
    rh[u] = r < s ? S.rho[r] : zero<A>();
  }
  if (tid < kBlkCols * kBlkCols) R1[tid] = B.R1[tid];
  if (tid == 0) cl = *S.ctrl;  // the control block, kept in LDS and written back
  int ph = 0;
  if (!mblk_cholqr<A, RPL>(X, nb, R2, gbuf)) mblk_qr<A, RPL>(X, nb, R2, scr, xs, nw, ph);
  __syncthreads();
  if (tid < kBlkCols * kBlkCols) {
    const int c = tid >> 3, b = tid & 7;
    A v = zero<A>();
    if (c <= b && b < nb)
      for (int e = c; e <= b; ++e) v += R2[e * kBlkCols + c] * R1[b * kBlkCols + e];
    RB[b * kBlkCols + c] = v;
  }
  __syncthreads();
  // The steps.  Every projection of the incoming residual in one sum, then
  // the residual left after each step in a second: the block's columns are
  // orthonormal, so projecting the incoming residual on column b equals
  // projecting what the steps before b left of it, up to rounding.  A step
  // with rank loss keeps its column out (projection 0).
  bool loss[kBlkCols];
#pragma unroll
  for (int b = 0; b < kBlkCols; ++b) loss[b] = b < nb && !(re(RB[b * kBlkCols + b]) > rank_rtol * n0s[b]);
  A zb[kBlkCols];
  {
    double d[kBlkCols * NC];
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) {
      A acc = zero<A>();
      if (b < nb && !loss[b]) {
#pragma unroll
        for (int u = 0; u < RPL; ++u) acc = fmac_conj(acc, X[b][u], rh[u]);
      }
      split_re(acc, d + b * NC);
    }
    grp_sums<kBlkCols * NC>(d, scr, xs, nw, ph);
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) join_re(zb[b], d + b * NC);
  }
  double nn[kBlkCols];
  {
    A rr[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) rr[u] = rh[u];
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b) {
      if (b < nb && !loss[b]) {
#pragma unroll
        for (int u = 0; u < RPL; ++u) rr[u] = fmsub(rr[u], X[b][u], zb[b]);
      }
      nn[b] = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) nn[b] += abs2(rr[u]);
    }
    grp_sums<kBlkCols>(nn, scr, xs, nw, ph);
  }
  if (mode != 0) {
    // recycled columns (the cycle's start): every column committed, its
    // projection of the residual recorded; after the last block, the
    // sketched residual over span(U) starts the residual control
#pragma unroll
    for (int b = 0; b < kBlkCols; ++b)
      if (b < nb && !loss[b]) {
#pragma unroll
        for (int u = 0; u < RPL; ++u) rh[u] = fmsub(rh[u], X[b][u], zb[b]);
      }
    if (tid < kBlkCols) {
      A zv = zb[0];
#pragma unroll
      for (int b = 1; b < kBlkCols; ++b)
        if (tid == b) zv = zb[b];
      if (tid < nb) S.z[col0 + tid] = zv;
    }
    if (mode == 2) {
      double q[1] = {0.0};
#pragma unroll
      for (int u = 0; u < RPL; ++u) q[0] += abs2(rh[u]);
      grp_sums<1>(q, scr, xs, nw, ph);
      if (tid == 0) {
        const double sres = sqrt(q[0]);
        S.sres_hist[0] = sres;
        control_start(S, col0 + nb, sres, gv);
      }
    }
    if (tid == 0) sh_halt = nb - 1;
  } else if (tid == 0) {
    // the residual control in step order, up to the step that halts
    A zs[kBlkCols];
    double ss[kBlkCols];
    int last = nb - 1, halted = 0;
#pragma unroll
    for (int bb = 0; bb < kBlkCols; ++bb) {
      zs[bb] = zb[bb];
      ss[bb] = sqrt(nn[bb]);
    }
#pragma unroll
    for (int bb = 0; bb < kBlkCols; ++bb) {
      if (bb >= nb || halted) continue;
      const int j = jb + bb, col = col0 + bb;
      const double sres = ss[bb];
      const bool brk = brks[bb];
      const int i0 = j - t > 0 ? j - t : 0, tw = j - i0;
      const double nuj = nujs[bb];
      S.nu[j] = nuj;
      for (int qq = 0; qq <= tw; ++qq) S.H[(int64_t)(j - 1) * S.ldh + i0 + qq] = hcs[bb * (kMaxWindow + 1) + qq];
      S.z[col] = zs[bb];
      int flags = 0;
      if (brk) flags |= 2;
      if (loss[bb]) flags |= 4;
      const bool due = control_due(&cl, sres);  // (updates the estimate: always evaluated)
      const bool halt = due || j == m || brk || loss[bb];
      if (halt) flags |= 1;
      S.sres_hist[j] = sres;
      if (halt) {
        S.ctrl->est = cl.est;
        S.ctrl->sprev = cl.sprev;
        S.ctrl->halt = 1;
        S.ctrl->halt_j = j;
        S.ctrl->flags = flags;
      }
      put_record(S, j, sres, nuj, flags, halt);
      if (halt) {
        last = bb;
        halted = 1;
      }
    }
    if (!halted) {
      S.ctrl->est = cl.est;
      S.ctrl->sprev = cl.sprev;
    }
    sh_halt = last;
  }
  __syncthreads();
  const int last = sh_halt;
  // the residual after the last finished step
#pragma unroll
  for (int b = 0; b < kBlkCols; ++b)
    if (mode == 0 && b <= last && b < nb && !loss[b]) {
#pragma unroll
      for (int u = 0; u < RPL; ++u) rh[u] = fmsub(rh[u], X[b][u], zb[b]);
    }
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int r = mblk_row<A, RPL>(u, nw);
    if (r < s) S.rho[r] = rh[u];
  }
  // commit Q and the block's R up to the last finished step
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int r = mblk_row<A, RPL>(u, nw);
    if (r < s) {
#pragma unroll
      for (int b = 0; b < kBlkCols; ++b)
        if (b <= last) S.Q[(int64_t)(col0 + b) * S.ldq + r] = X[b][u];
    }
  }
  if (tid < kBlkCols * kBlkCols) {
    const int c = tid >> 3, b = tid & 7;
    if (c <= b && b <= last) S.R[(int64_t)(col0 + b) * S.ldr + col0 + c] = RB[b * kBlkCols + c];
  }
}

// Rows per lane of the in-block kernels and their waves for a sketch of s
// rows: the smallest RPL that kMblkMaxWaves waves cover (the block, the
// Gram products and the fallback's sums stay in registers), then the fewest
// waves for it; false when s exceeds kMblkMaxWaves waves of the largest RPL.
template <class A>
static bool mblk_shape(int s, int* rpl, int* nw) {
  constexpr int opts[3] = {2, 4, sizeof(A) == 16 ? 4 : 8};
  if (s < 1) return false;
  for (int o : opts)
    if (s <= 64 * kMblkMaxWaves * o) {
      *rpl = o;
      *nw = (s + 64 * o - 1) / (64 * o);
      return true;
    }
  return false;
}

// The in-block factorisation, the second sweep and the finish of one block.
template <class A, int RPL>
static void launch_mblk_tail(hipStream_t st, const LsqState<A>& S, int jb, int nb, int m, int t, int s, int col0,
                             int nw, double rank_rtol, int mode = 0, GivensInit gv = GivensInit{}) {
  const size_t lds_upd = (size_t)kMblkSweepWaves * kBlkCols * 64 * sizeof(A);
  hipLaunchKernelGGL((k_mblk_qr<A, RPL>), dim3(1), dim3(64 * nw), 0, st, S, nb, s);
  if (col0 > 0) {
    hipLaunchKernelGGL(k_mblk_proj<A>, dim3((col0 + 7) / 8), dim3(kMblkSweepThreads), 0, st, S.Q, S.ldq, col0, s,
                       S.bw.W, nb, S.bw.P, S.R + (int64_t)col0 * S.ldr, S.ldr, (const A*)S.bw.R1, S.ctrl);
    hipLaunchKernelGGL(k_mblk_upd<A>, dim3((s + 63) / 64), dim3(kMblkSweepThreads), lds_upd, st, S.Q, S.ldq, col0,
                       s, S.bw.W, nb, S.bw.P, S.ctrl);
  }
  hipLaunchKernelGGL((k_mblk_fin<A, RPL>), dim3(1), dim3(64 * nw), 0, st, S, jb, nb, m, t, s, col0, rank_rtol,
                     mode, gv);
}

// The several-workgroup block path for steps j0 .. j1 (false: the sketch is
// too long for the in-block kernels' registers).
template <class A>
static bool launch_lsq_blocks_multi(hipStream_t st, LsqState<A> S, int j0, int j1, int khat, int m, int t, int s,
                                    const A* redb, int64_t slotr, int nslot, double brtol, double rank_rtol) {
  constexpr bool cpx = sizeof(A) == 16;
  int rpl = 0, nw = 0;
  if (!mblk_shape<A>(s, &rpl, &nw)) return false;
  const size_t lds_upd = (size_t)kMblkSweepWaves * kBlkCols * 64 * sizeof(A);
  for (int jb = j0; jb <= j1; jb += kBlkCols) {
    const int nb = std::min(kBlkCols, j1 - jb + 1);
    const int col0 = khat + jb - 1;  // committed columns of Q
    hipLaunchKernelGGL(k_mblk_head<A>, dim3(1), dim3(std::min(kMblkHeadThreads, (s + 63) / 64 * 64)), 0, st, S, jb,
                       nb, khat, t, s, redb, slotr, nslot, brtol);
    if (col0 > 0) {
      hipLaunchKernelGGL(k_mblk_proj<A>, dim3((col0 + 7) / 8), dim3(kMblkSweepThreads), 0, st, S.Q, S.ldq, col0,
                         s, S.bw.W, nb, S.bw.P, S.R + (int64_t)col0 * S.ldr, S.ldr, (const A*)nullptr, S.ctrl);
      hipLaunchKernelGGL(k_mblk_upd<A>, dim3((s + 63) / 64), dim3(kMblkSweepThreads), lds_upd, st, S.Q, S.ldq,
                         col0, s, S.bw.W, nb, S.bw.P, S.ctrl);
    }
    if (rpl == 2) launch_mblk_tail<A, 2>(st, S, jb, nb, m, t, s, col0, nw, rank_rtol);
    else if (rpl == 4 || cpx) launch_mblk_tail<A, 4>(st, S, jb, nb, m, t, s, col0, nw, rank_rtol);
    else if constexpr (!cpx) launch_mblk_tail<A, 8>(st, S, jb, nb, m, t, s, col0, nw, rank_rtol);
  }
  return true;
}

// The cycle start on the several-workgroup block path: the khat recycled
// columns of SAW appended to the factor in blocks of up to 8 (the same
// projections, updates and in-block factorisations as the steps), z and the
// projected residual from S r0, the sketched residual over span(U) and the
// control's start (false: the sketch is too long for the in-block kernels).
template <class A>
static bool launch_lsq_init_multi(hipStream_t st, LsqState<A> S, int khat, int s, const A* Sr, double rank_rtol,
                                  GivensInit gv) {
  constexpr bool cpx = sizeof(A) == 16;
  int rpl = 0, nw = 0;
  if (khat < 1 || !mblk_shape<A>(s, &rpl, &nw)) return false;
  const size_t lds_upd = (size_t)kMblkSweepWaves * kBlkCols * 64 * sizeof(A);
  for (int c0 = 0; c0 < khat; c0 += kBlkCols) {
    const int nb = std::min(kBlkCols, khat - c0);
    const int mode = c0 + nb == khat ? 2 : 1;
    hipLaunchKernelGGL(k_mblk_init_head<A>, dim3(1), dim3(std::min(kMblkHeadThreads, (s + 63) / 64 * 64)), 0, st,
                       S, c0, nb, s, Sr);
    if (c0 > 0) {
      hipLaunchKernelGGL(k_mblk_proj<A>, dim3((c0 + 7) / 8), dim3(kMblkSweepThreads), 0, st, S.Q, S.ldq, c0, s,
                         S.bw.W, nb, S.bw.P, S.R + (int64_t)c0 * S.ldr, S.ldr, (const A*)nullptr, S.ctrl);
      hipLaunchKernelGGL(k_mblk_upd<A>, dim3((s + 63) / 64), dim3(kMblkSweepThreads), lds_upd, st, S.Q, S.ldq, c0,
                         s, S.bw.W, nb, S.bw.P, S.ctrl);
    }
    if (rpl == 2) launch_mblk_tail<A, 2>(st, S, 0, nb, 0, 0, s, c0, nw, rank_rtol, mode, gv);
    else if (rpl == 4 || cpx) launch_mblk_tail<A, 4>(st, S, 0, nb, 0, 0, s, c0, nw, rank_rtol, mode, gv);
    else if constexpr (!cpx) launch_mblk_tail<A, 8>(st, S, 0, nb, 0, 0, s, c0, nw, rank_rtol, mode, gv);
  }
  return true;
}

// LDS of the batched kernel: update partials, reduction scratch, window ring
template <class A>
static constexpr size_t lsq_steps_lds(int rl, int cw) {
  return (size_t)kRegWaves * 64 * rl * sizeof(A) +
         (size_t)kRegWaves * 16 * (cw * (sizeof(A) / 8) + 1) * 8 + (size_t)kMaxWindow * 64 * rl * sizeof(A);
}

#define SDR_LSQ_STEPS_CASE(RL, CW)                                                            \
  if constexpr (lsq_steps_lds<A>(RL, CW) <= 64 * 1024 && (sizeof(A) == 8 || CW == 8)) {        \
    if (rl == RL && cw == CW) {                                                               \
      hipLaunchKernelGGL((k_lsq_steps_reg<A, RL, CW>), dim3(1), dim3(kLsqBlock), 0, st, S, j0, \
                         j1, khat, m, t, s, redb, slotr, nslot, brtol, rank_rtol);             \
      return;                                                                                 \
    }                                                                                         \
  }

template <class A>
void launch_lsq_steps(hipStream_t st, LsqState<A> S, int j0, int j1, int khat, int m, int t, int s,
                      const A* redb, int64_t slotr, int nslot, double brtol, double rank_rtol, int kind) {
  int rl = 0, cw = 0;
  if (kind == 0 && lsq_reg_shape<A>(s, khat + m + 1, &rl, &cw)) {
    SDR_LSQ_STEPS_CASE(2, 8)
    SDR_LSQ_STEPS_CASE(2, 16)
    SDR_LSQ_STEPS_CASE(4, 16)
    SDR_LSQ_STEPS_CASE(4, 8)
  }
  if ((kind == 0 || kind == 3) &&
      launch_lsq_blocks_multi<A>(st, S, j0, j1, khat, m, t, s, redb, slotr, nslot, brtol, rank_rtol))
    return;
  if (kind == 0 || kind == 1) {
    size_t lds = 0;
    const int prow = (std::max(1, khat + j1 - 1) + 7) / 8 * 8;  // P rows padded to whole groups
    const int bc = lsq_block_cols<A>(s, prow, &lds);
    if (bc > 0) {
      hipLaunchKernelGGL(k_lsq_block<A>, dim3(1), dim3(kBlkThreads), lds, st, S, j0, j1, khat, m, t, s, redb,
                         slotr, nslot, brtol, rank_rtol, bc, prow);
      return;
    }
  }
  // shapes without a batched kernel: one launch per step
  for (int j = j0; j <= j1; ++j)
    launch_lsq_step<A>(st, S, j, khat, m, t, s, redb + slotr * (j % nslot), brtol, rank_rtol);
}

template <class A>
__global__ __launch_bounds__(kLsqBlock) void k_lsq_init(LsqState<A> S, int khat, int s,
                                                        const A* __restrict__ Sr, double rank_rtol,
                                                        GivensInit gv) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lmax = khat + 1;
  const int ch = lsq_chunk<A>(s, lmax);
  A* a = reinterpret_cast<A*>(smem_raw);
  A* accb = a + s;
  A* cbuf = accb + s;
  A* qs = cbuf + 2 * lmax;
  __shared__ A red[kLsqBlock / 64];
  for (int r = threadIdx.x; r < s; r += blockDim.x) S.rho[r] = Sr[r];
  __syncthreads();
  double sres = 0.0;
  for (int c = 0; c < khat; ++c) {
    for (int r = threadIdx.x; r < s; r += blockDim.x) a[r] = S.SAW[(int64_t)c * S.ldsaw + r];
    __syncthreads();
    bool loss = false;
    sres = qr_append(S, a, accb, cbuf, qs, ch, red, c, s, rank_rtol, &loss);
  }
  if (khat == 0) sres = rho_norm(S.rho, s, (double*)red);
  if (threadIdx.x == 0) {
    S.sres_hist[0] = sres;
    control_start(S, khat, sres, gv);
  }
}

template <class A>
void launch_lsq_init(hipStream_t st, LsqState<A> S, int khat, int s, const A* Sr, double rank_rtol,
                     int m, GivensInit gv, int kind) {
  int rl = 0, cw = 0;
  // the same register shape as the step kernel of this cycle
  if (kind == 0 && lsq_reg_shape<A>(s, khat + m + 1, &rl, &cw)) {
    SDR_LSQ_REG_CASE(2, 8, k_lsq_init_reg, S, khat, s, Sr, rank_rtol, gv)
    SDR_LSQ_REG_CASE(2, 16, k_lsq_init_reg, S, khat, s, Sr, rank_rtol, gv)
    SDR_LSQ_REG_CASE(4, 16, k_lsq_init_reg, S, khat, s, Sr, rank_rtol, gv)
    SDR_LSQ_REG_CASE(4, 8, k_lsq_init_reg, S, khat, s, Sr, rank_rtol, gv)
  }
  // the several-workgroup block path, where the steps take it too
  if ((kind == 0 || kind == 3) && launch_lsq_init_multi<A>(st, S, khat, s, Sr, rank_rtol, gv)) return;
  const int lmax = khat + 1;
  const size_t lds = (size_t)(2 * s + 2 * lmax + lsq_chunk<A>(s, lmax) * s) * sizeof(A);
  hipLaunchKernelGGL(k_lsq_init<A>, dim3(1), dim3(kLsqBlock), lds, st, S, khat, s, Sr, rank_rtol, gv);
}

// R y = z by columns (back substitution), then the basis coefficients.
template <class A>
__global__ __launch_bounds__(kLsqBlock) void k_backsolve(LsqState<A> S, int n, int khat,
                                                         A* __restrict__ ycoef) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  A* y = reinterpret_cast<A*>(smem_raw);
  for (int i = threadIdx.x; i < n; i += blockDim.x) y[i] = S.z[i];
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const A rii = S.R[(int64_t)i * S.ldr + i];
      const double d = abs2(rii);
      if (d > 0.0) {
        // y_i / r_ii = y_i * conj(r_ii) / |r_ii|^2
        y[i] = scale(y[i] * conj(rii), 1.0 / d);
      } else {
        y[i] = zero<A>();
      }
    }
    __syncthreads();
    const A yi = y[i];
    for (int k = threadIdx.x; k < i; k += blockDim.x) y[k] -= S.R[(int64_t)i * S.ldr + k] * yi;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    ycoef[i] = i < khat ? y[i] : scale(y[i], 1.0 / S.nu[i - khat]);
}

template <class A>
void launch_backsolve(hipStream_t st, LsqState<A> S, int n, int khat, A* ycoef) {
  hipLaunchKernelGGL(k_backsolve<A>, dim3(1), dim3(kLsqBlock), (size_t)n * sizeof(A), st, S, n,
                     khat, ycoef);
}

// -------------------------------------------------------- batched sketch ---
template <class X>
__global__ __launch_bounds__(kBlock) void k_sketch_cols(int n, const X* __restrict__ x, int64_t ld,
                                                        int cc, SketchSpec sk,
                                                        typename traits<X>::acc* __restrict__ part,
                                                        int nb) {
  using A = typename traits<X>::acc;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  A* acc = reinterpret_cast<A*>(smem_raw);  // [kWaves][cc * s]
  __shared__ A red[kWaves];
  const int s = sk.s;
  const int w = cc * s;
  for (int i = threadIdx.x; i < kWaves * w; i += kBlock) acc[i] = zero<A>();
  __syncthreads();
  A* mine = acc + (threadIdx.x >> 6) * w;
  double nrm[8];
  for (int c = 0; c < 8; ++c) nrm[c] = 0.0;
  const int r0 = blockIdx.x * kRowsUpdate;
  const int r1 = min(n, r0 + kRowsUpdate);
  for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
    const uint64_t base = sk.seed + kGamma * ((uint64_t)r * (uint64_t)sk.words + 1ull);
    for (int g = 0; g < sk.words; ++g) {
      const uint64_t h = mix64(base + (uint64_t)g * kGamma);
      for (int q = 0; q < 4; ++q) {
        const int b = 4 * g + q;
        if (b < sk.zeta) {
          const uint32_t u = (uint32_t)(h >> (16 * q)) & 0xFFFFu;
          const int row = b * sk.bsz + (int)(((u >> 1) * (uint32_t)sk.bsz) >> 15);
          const bool ng = (u & 1u) != 0u;
          for (int c = 0; c < cc; ++c) lds_add(&mine[c * s + row], neg_if(widen(x[r + c * ld]), ng));
        }
      }
    }
    for (int c = 0; c < cc; ++c) nrm[c] += abs2(widen(x[r + c * ld]));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < w; i += kBlock) {
    A sum = acc[i];
    for (int q = 1; q < kWaves; ++q) sum += acc[q * w + i];
    part[(int64_t)i * nb + blockIdx.x] = sum;
  }
  for (int c = 0; c < cc; ++c) {
    const double ns = block_sum(nrm[c], (double*)red);
    if (threadIdx.x == 0) {
      A v = zero<A>();
      *(double*)&v = ns;
      part[(int64_t)(w + c) * nb + blockIdx.x] = v;
    }
  }
}

template <class X>
void launch_sketch_cols(hipStream_t st, int n, const X* x, int64_t ld, int cc, SketchSpec sk,
                        typename traits<X>::acc* part, int nb) {
  using A = typename traits<X>::acc;
  const size_t lds = (size_t)kWaves * cc * sk.s * sizeof(A);
  hipLaunchKernelGGL(k_sketch_cols<X>, dim3(nb), dim3(kBlock), lds, st, n, x, ld, cc, sk, part, nb);
}

// ----------------------------------- subsampled randomised DCT sketch ---
// y_i = a_i sum_r e_r x_r cos(pi p_i (2r + 1) / (2N)) over a tile of
// kRowsSpmv rows per block of kDctThreads: the tile's e_r x_r is staged in
// LDS (and a copy with every other entry negated, for the alternating form).
// Each half of the block takes half of the tile's rows; thread f of a half
// owns kept rows f, f + kBlock, ...  Each half runs its rows as two chains of
// kDctChain entries, each started from its phase pi p (2 r + 1) / (2N)
// reduced exactly in integers (mod 4N) and advanced by Reinsch's recurrence:
// per entry and kept row one multiply-add into the sum and two recurrence
// operations (error O(kDctChain eps)).  The halves' sums are added in a fixed
// order.  ALU-bound: s multiply-adds per entry.
constexpr int kDctThreads = 2 * kBlock;
constexpr int kDctChain = kRowsSpmv / 4;  // 384 (even: chains start on even entries)
constexpr int kDctMaxFpt = 8;             // kept rows per thread (s <= 2048)

// cos(phi) and the first difference d = c_0 - c_{-1} of the row's recurrence.
__device__ __forceinline__ void dct_start(const DctRow& w, uint64_t ph, double ang, double* c, double* d) {
  double sn, cs;
  sincos((double)ph * ang, &sn, &cs);
  *c = cs;
  // mode 0: c_q = cos(phi + q b): d = cos phi - cos(phi - b) = -2 sin(b/2) sin(phi - b/2)
  // mode 1: c'_q = cos(phi - q b'): d = cos phi - cos(phi + b') = 2 sin(b'/2) sin(phi + b'/2)
  *d = w.mode ? 2.0 * w.sh * (sn * w.ch + cs * w.sh) : -2.0 * w.sh * (sn * w.ch - cs * w.sh);
}

template <class X>
__global__ __launch_bounds__(kDctThreads) void k_dct_sketch(int n, const X* __restrict__ x, DctSpec d,
                                                            typename traits<X>::acc* __restrict__ part,
                                                            int nb, int with_norm,
                                                            const Ctrl* __restrict__ ctrl) {
  using A = typename traits<X>::acc;
  if (ctrl && ctrl->halt) return;
  __shared__ A vb[2 * kRowsSpmv + 1];  // e x, then (-1)^q e x (one pad entry between: other banks)
  __shared__ double red[kDctThreads / 64];
  A* v0 = vb;
  A* v1 = vb + kRowsSpmv + 1;
  const int tile = xcd_tile(blockIdx.x, nb);
  const int r0 = tile * kRowsSpmv;
  const int len = min(kRowsSpmv, n - r0);
  double nx = 0.0;
  for (int q = (int)threadIdx.x; q < kRowsSpmv; q += kDctThreads) {
    A e = zero<A>();
    if (q < len) {
      const int r = r0 + q;
      const A xv = widen(x[r]);
      nx += abs2(xv);
      const uint64_t h = mix64(d.sign_seed + kGamma * (uint64_t)(r + 1));
      e = neg_if(xv, (h & 1ull) != 0ull);
    }
    v0[q] = e;
    v1[q] = neg_if(e, (q & 1) != 0);
  }
  __syncthreads();
  const int half = (int)threadIdx.x / kBlock, lt = (int)threadIdx.x % kBlock;
  // this half's chains: [qa, qa + na) and [qb, qb + nbb)
  const int qa = half * 2 * kDctChain, qb = qa + kDctChain;
  const int na = max(0, min(kDctChain, len - qa)), nbb = max(0, min(kDctChain, len - qb));
  const int fpt = (d.s + kBlock - 1) / kBlock;
  const uint64_t n4 = (uint64_t)d.n4;
  A acc[kDctMaxFpt];
#pragma unroll
  for (int k = 0; k < kDctMaxFpt; ++k) {
    acc[k] = zero<A>();
    const int f = lt + k * kBlock;
    if (k >= fpt || f >= d.s || na == 0) continue;
    const DctRow w = d.rows[f];
    const A* vs = w.mode ? v1 : v0;
    double ca, da, cb, db;
    dct_start(w, ((uint64_t)w.p * (uint64_t)(2 * (r0 + qa) + 1)) % n4, d.ang, &ca, &da);
    dct_start(w, ((uint64_t)w.p * (uint64_t)(2 * (r0 + qb) + 1)) % n4, d.ang, &cb, &db);
    const double lam = w.lam;
    A sa = zero<A>(), sb = zero<A>();
    const A* pa = vs + qa;
    const A* pb = vs + qb;
    int q = 0;
    for (; q + 2 <= nbb; q += 2) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        sa += pa[q + u] * ca;
        da -= lam * ca;
        ca += da;
        sb += pb[q + u] * cb;
        db -= lam * cb;
        cb += db;
      }
    }
    for (; q < nbb; ++q) {
      sa += pa[q] * ca;
      da -= lam * ca;
      ca += da;
      sb += pb[q] * cb;
      db -= lam * cb;
      cb += db;
    }
    for (; q < na; ++q) {
      sa += pa[q] * ca;
      da -= lam * ca;
      ca += da;
    }
    acc[k] = sa + sb;
  }
  // the halves' sums, added in a fixed order (half 0, then half 1)
  const double tn = with_norm ? block_sum(nx, red) : 0.0;  // (its barriers also end the reads of vb)
  if (!with_norm) __syncthreads();
#pragma unroll
  for (int k = 0; k < kDctMaxFpt; ++k) {
    if (k >= fpt) break;
    if (half == 1) vb[lt] = acc[k];
    __syncthreads();
    const int f = lt + k * kBlock;
    if (half == 0 && f < d.s) {
      const DctRow& w = d.rows[f];
      part[(int64_t)w.out * nb + tile] = scale(acc[k] + vb[lt], w.a);
    }
    __syncthreads();
  }
  if (with_norm && threadIdx.x == 0) put_re(&part[(int64_t)d.s * nb + tile], tn);
}

template <class X>
void launch_dct_sketch(hipStream_t st, int n, const X* x, DctSpec d, typename traits<X>::acc* part, int nb,
                       bool with_norm, const Ctrl* ctrl, hipEvent_t e0, hipEvent_t e1) {
  if (e0)
    hipExtLaunchKernelGGL(k_dct_sketch<X>, dim3(nb), dim3(kDctThreads), 0, st, e0, e1, 0, n, x, d, part, nb,
                          with_norm ? 1 : 0, ctrl);
  else
    hipLaunchKernelGGL(k_dct_sketch<X>, dim3(nb), dim3(kDctThreads), 0, st, n, x, d, part, nb,
                       with_norm ? 1 : 0, ctrl);
}

// ------------------------------------------------- tall-skinny products ---
// acc + sum_i X(r, i) y_i over nc columns, in column order, eight loads in
// flight per round.
template <class T, class A>
__device__ __forceinline__ A dot_cols(const T* __restrict__ X, int64_t ld, int nc, const A* ys, int r, A acc) {
  int i = 0;
  for (; i + 8 <= nc; i += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = X[r + (int64_t)(i + u) * ld];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += widen(v[u]) * ys[i + u];
  }
  for (; i < nc; ++i) acc += widen(X[r + (int64_t)i * ld]) * ys[i];
  return acc;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_gemv_basis(int n, const T* __restrict__ U, int64_t ldu,
                                                       int ku, const T* __restrict__ P, int64_t ldp,
                                                       int jp, const typename traits<T>::acc* __restrict__ y,
                                                       typename traits<T>::acc* __restrict__ out) {
  using A = typename traits<T>::acc;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  A* ys = reinterpret_cast<A*>(smem_raw);
  for (int i = threadIdx.x; i < ku + jp; i += blockDim.x) ys[i] = y[i];
  __syncthreads();
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    A acc = zero<A>();
    acc = dot_cols(U, ldu, ku, ys, r, acc);
    acc = dot_cols(P, ldp, jp, ys + ku, r, acc);
    out[r] = acc;
  }
}

template <class T>
void launch_gemv_basis(hipStream_t st, int n, const T* U, int64_t ldu, int ku, const T* P,
                       int64_t ldp, int jp, const typename traits<T>::acc* y,
                       typename traits<T>::acc* out) {
  using A = typename traits<T>::acc;
  const int nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_gemv_basis<T>, dim3(nb), dim3(kBlock), (size_t)(ku + jp) * sizeof(A), st, n,
                     U, ldu, ku, P, ldp, jp, y, out);
}

// End of a residual kernel: with the sketch (sk.s > 0), the per-wave bins
// summed over the waves into partial rows 0 .. s-1 and ||rnew||^2 into row
// s, the layout and order of k_sketch_cols for one column; without it,
// ||rnew||^2 into row 0.
template <class A>
__device__ __forceinline__ void store_residual_partials(A* __restrict__ part, int s, double nrm,
                                                        const A* bins_all, A* red, int tile) {
  const double sum = block_sum(nrm, (double*)red);  // (its barriers also complete the bins)
  for (int i = threadIdx.x; i < s; i += kBlock) {
    A t = bins_all[i];
    for (int q = 1; q < kWaves; ++q) t += bins_all[q * s + i];
    part[(int64_t)i * gridDim.x + tile] = t;
  }
  if (threadIdx.x == 0) {
    A v = zero<A>();
    *(double*)&v = sum;
    part[(int64_t)s * gridDim.x + tile] = v;
  }
}

// rnew = r0 - A x over CSR (full-precision values), partial ||rnew||^2 per
// row tile; with sk.s > 0 also the partial sketch of rnew, so that the next
// cycle's S r0 needs no pass of its own.
template <class A>
__global__ __launch_bounds__(kBlock) void k_spmv_residual(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci,
                                                          const A* __restrict__ val,
                                                          const A* __restrict__ x,
                                                          const A* __restrict__ r0,
                                                          A* __restrict__ rnew, A* __restrict__ part,
                                                          SketchSpec sk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ A red[kWaves];
  const int s = sk.s;
  A* bins_all = reinterpret_cast<A*>(smem_raw);
  A* bins = bins_all + (threadIdx.x >> 6) * s;
  for (int i = threadIdx.x & 63; i < s; i += 64) bins[i] = zero<A>();
  double nrm = 0.0;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);  // partial sums are stored by tile
  const int b0 = tile * kRowsUpdate;
  const int b1 = min(n, b0 + kRowsUpdate);
  for (int r = b0 + (int)threadIdx.x; r < b1; r += kBlock) {
    A acc = zero<A>();
    const int e1 = rp[r + 1];
    for (int e = rp[r]; e < e1; ++e) acc += val[e] * x[ci[e]];
    const A v = r0[r] - acc;
    rnew[r] = v;
    if (s > 0) sketch_scatter(bins, r, v, sk);
    nrm += abs2(v);
  }
  store_residual_partials(part, s, nrm, bins_all, red, tile);
}

// rnew = r0 - A x over the diagonal storage (values in the accumulation
// type); partials as k_spmv_residual.
template <class A, int ND>
__global__ __launch_bounds__(kBlock) void k_spmv_dia_residual(int n, DiaView<A> M, const A* __restrict__ x,
                                                              const A* __restrict__ r0,
                                                              A* __restrict__ rnew, A* __restrict__ part,
                                                              SketchSpec sk) {
  constexpr int KD = ND > 0 ? ND : kMaxDiag;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ A red[kWaves];
  const int s = sk.s;
  A* bins_all = reinterpret_cast<A*>(smem_raw);
  A* bins = bins_all + (threadIdx.x >> 6) * s;
  for (int i = threadIdx.x & 63; i < s; i += 64) bins[i] = zero<A>();
  const int nd = ND > 0 ? ND : M.ndiag;
  double nrm = 0.0;
  // tiles XCD-aware, so that the +-n halo rows of x are in the L2 of the
  // XCD that works on the neighbouring tiles
  const int tile = xcd_tile(blockIdx.x, gridDim.x);  // partial sums are stored by tile
  const int b0 = tile * kRowsUpdate;
  const int b1 = min(n, b0 + kRowsUpdate);
  for (int r = b0 + (int)threadIdx.x; r < b1; r += kBlock) {
    A vv[KD], xc[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) {
      if (ND > 0 || k < nd) {
        vv[k] = M.val[(int64_t)k * n + r];
        xc[k] = x[min(max(r + M.off[k], 0), n - 1)];
      }
    }
    const A rr = r0[r];
    A acc = zero<A>();
#pragma unroll
    for (int k = 0; k < KD; ++k) {
      if (ND > 0 || k < nd) {
        const int c = r + M.off[k];
        const A t = vv[k] * xc[k];
        acc += (c >= 0 && c < n) ? t : zero<A>();
      }
    }
    const A v = rr - acc;
    rnew[r] = v;
    if (s > 0) sketch_scatter(bins, r, v, sk);
    nrm += abs2(v);
  }
  store_residual_partials(part, s, nrm, bins_all, red, tile);
}

template <class A>
void launch_spmv_dia_residual(hipStream_t st, int n, DiaView<A> M, const A* x, const A* r0, A* rnew, A* part,
                              int nb, SketchSpec sk) {
  void (*kern)(int, DiaView<A>, const A*, const A*, A*, A*, SketchSpec);
  switch (M.ndiag) {
    case 3: kern = k_spmv_dia_residual<A, 3>; break;
    case 5: kern = k_spmv_dia_residual<A, 5>; break;
    case 7: kern = k_spmv_dia_residual<A, 7>; break;
    case 9: kern = k_spmv_dia_residual<A, 9>; break;
    default: kern = k_spmv_dia_residual<A, 0>; break;
  }
  const size_t lds = (size_t)kWaves * sk.s * sizeof(A);
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), lds, st, n, M, x, r0, rnew, part, sk);
}

template <class A>
void launch_spmv_residual(hipStream_t st, int n, const int* rp, const int* ci, const A* val,
                          const A* x, const A* r0, A* rnew, A* part, int nb, SketchSpec sk) {
  const size_t lds = (size_t)kWaves * sk.s * sizeof(A);
  hipLaunchKernelGGL(k_spmv_residual<A>, dim3(nb), dim3(kBlock), lds, st, n, rp, ci, val, x, r0, rnew,
                     part, sk);
}

// C = [U P] G, one row per thread with KM accumulators.  G is row major (row
// stride ldg, zero beyond column kc): its entries are the same for every
// lane, so they are read with scalar loads straight into the multiply-adds'
// scalar operands (a row of G in a few wide loads, no LDS traffic).
template <class T, int KM>
__global__ __launch_bounds__(kBlock) void k_gemm_basis(int n, const T* __restrict__ U, int64_t ldu,
                                                       int ku, const T* __restrict__ P, int64_t ldp,
                                                       int jp, const typename traits<T>::acc* __restrict__ G,
                                                       int ldg, int kc, T* __restrict__ C, int64_t ldc) {
  using A = typename traits<T>::acc;
  const int l0 = ku + jp;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    A acc[KM];
#pragma unroll
    for (int c = 0; c < KM; ++c) acc[c] = zero<A>();
    // two input columns per round, their loads issued together (the column
    // pointer is chosen without a branch); accumulation in column order.
    // Wider rounds hold more rows of G in scalar registers than fit and ran
    // slower.
    int i = 0;
    for (; i + 2 <= l0; i += 2) {
      A v[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ii = i + u;
        const T* src = ii < ku ? U + ii * ldu : P + (int64_t)(ii - ku) * ldp;
        v[u] = widen(src[r]);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const A* g = G + (int64_t)(i + u) * ldg;
#pragma unroll
        for (int c = 0; c < KM; ++c) acc[c] += v[u] * g[c];
      }
    }
    for (; i < l0; ++i) {
      const T* src = i < ku ? U + i * ldu : P + (int64_t)(i - ku) * ldp;
      const A v = widen(src[r]);
      const A* g = G + (int64_t)i * ldg;
#pragma unroll
      for (int c = 0; c < KM; ++c) acc[c] += v * g[c];
    }
#pragma unroll
    for (int c = 0; c < KM; ++c)
      if (c < kc) C[r + c * ldc] = narrow<T>(acc[c]);
  }
}

// Real data: two adjacent rows per thread, one two-wide load per column, so
// each scalar entry of G feeds two multiply-adds and fewer rows of G are held
// at once (no scalar-register spills at KM <= 24).  Each row's sum is formed
// in column order as in k_gemm_basis, with the same bits.  Requires n, the
// leading dimensions and the base addresses even (two-element aligned).
template <class T> struct pair2;
template <> struct pair2<double> { using type = double2; };
template <> struct pair2<float> { using type = float2; };

template <class T, int KM>
__global__ __launch_bounds__(kBlock) void k_gemm_basis2(int n, const T* __restrict__ U, int64_t ldu,
                                                        int ku, const T* __restrict__ P, int64_t ldp,
                                                        int jp, const double* __restrict__ G, int ldg,
                                                        int kc, T* __restrict__ C, int64_t ldc) {
  using T2 = typename pair2<T>::type;
  const int l0 = ku + jp;
  // one pass: the grid covers the rows (a loop over the grid kept more
  // scalar registers live and spilled)
  const int r = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
  if (r >= n) return;
  {
    double a0[KM], a1[KM];
#pragma unroll
    for (int c = 0; c < KM; ++c) {
      a0[c] = 0.0;
      a1[c] = 0.0;
    }
    int i = 0;
    for (; i + 2 <= l0; i += 2) {
      T2 v[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ii = i + u;
        const T* src = ii < ku ? U + ii * ldu : P + (int64_t)(ii - ku) * ldp;
        v[u] = *reinterpret_cast<const T2*>(src + r);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const double* g = G + (int64_t)(i + u) * ldg;
        const double x0 = widen(v[u].x), x1 = widen(v[u].y);
#pragma unroll
        for (int c = 0; c < KM; ++c) {
          a0[c] += x0 * g[c];
          a1[c] += x1 * g[c];
        }
      }
    }
    for (; i < l0; ++i) {
      const T* src = i < ku ? U + i * ldu : P + (int64_t)(i - ku) * ldp;
      const T2 v = *reinterpret_cast<const T2*>(src + r);
      const double* g = G + (int64_t)i * ldg;
      const double x0 = widen(v.x), x1 = widen(v.y);
#pragma unroll
      for (int c = 0; c < KM; ++c) {
        a0[c] += x0 * g[c];
        a1[c] += x1 * g[c];
      }
    }
#pragma unroll
    for (int c = 0; c < KM; ++c)
      if (c < kc) {
        T2 o;
        o.x = narrow<T>(a0[c]);
        o.y = narrow<T>(a1[c]);
        *reinterpret_cast<T2*>(C + r + c * ldc) = o;
      }
  }
}

// C = [U P] G on the matrix cores (v_mfma_f64_16x16x4f64: a 16 x 4 block of
// A times a 4 x 16 block of B added to a 16 x 16 block, 64 lanes).  G, l0 x
// kc (l0 = ku + jp), is staged once per workgroup into LDS, as real and
// imaginary planes of W = 16 NCT columns (zero padded to a multiple of 4 rows
// and to W columns); the grid is persistent, each workgroup taking blocks of
// 512 rows, each wave 64 rows (four 16-row tiles).  Lane (i, q) = (lane % 16,
// lane / 16) supplies row i, basis column k0 + q of A and row k0 + q, column
// i of B; its result register v holds row 4 v + q, column i of the 16 x 16
// block (the layout measured on gfx950).
// A complex product takes four real ones: re += a.x g.x + a.y (-g.y),
// im += a.x g.y + a.y g.x.  The next four basis columns are loaded while the
// current ones are multiplied.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kGemmMfmaThreads = 512;
constexpr int kGemmMfmaRows = 64 * (kGemmMfmaThreads / 64);  // rows per workgroup block

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ double cre(double a) { return a; }
__device__ __forceinline__ double cim(double) { return 0.0; }
__device__ __forceinline__ double cre(cx<double> a) { return a.x; }
__device__ __forceinline__ double cim(cx<double> a) { return a.y; }

template <class T, int NCT>
__global__ __launch_bounds__(kGemmMfmaThreads) void k_gemm_basis_mfma(
    int n, const T* __restrict__ U, int64_t ldu, int ku, const T* __restrict__ P, int64_t ldp, int jp,
    const typename traits<T>::acc* __restrict__ G, int ldg, int kc, T* __restrict__ C, int64_t ldc) {
  using A = typename traits<T>::acc;
  constexpr bool CPX = traits<T>::cpx;
  constexpr int W = 16 * NCT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* gr = reinterpret_cast<double*>(smem_raw);
  const int l0 = ku + jp, l0p = (l0 + 3) & ~3;
  double* gi = gr + (size_t)l0p * W;
  for (int e = threadIdx.x; e < l0p * W; e += blockDim.x) {
    const int k = e / W, j = e - k * W;
    const A g = (k < l0 && j < kc) ? G[(int64_t)k * ldg + j] : zero<A>();
    gr[e] = cre(g);
    if constexpr (CPX) gi[e] = cim(g);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  for (int rb = blockIdx.x; (int64_t)rb * kGemmMfmaRows < n; rb += gridDim.x) {
    const int row0 = rb * kGemmMfmaRows + wv * 64;
    v4d acc[4][NCT][CPX ? 2 : 1];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int h = 0; h < (CPX ? 2 : 1); ++h) acc[t][ct][h] = v4d{0.0, 0.0, 0.0, 0.0};
    auto load = [&](int k0, A (&a)[4]) {
      const int c = k0 + q;
      const T* col = c < ku ? U + (int64_t)c * ldu : P + (int64_t)(c < l0 ? c - ku : 0) * ldp;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = row0 + t * 16 + i16;
        const A v = widen(col[min(r, n - 1)]);
        a[t] = (c < l0 && r < n) ? v : zero<A>();
      }
    };
    A an[4];
    load(0, an);
    for (int k0 = 0; k0 < l0p; k0 += 4) {
      A a[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = an[t];
      if (k0 + 4 < l0p) load(k0 + 4, an);
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const int e = (k0 + q) * W + ct * 16 + i16;
        const double br = gr[e];
        if constexpr (CPX) {
          const double bi = gi[e];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            acc[t][ct][0] = mfma_f64(cre(a[t]), br, acc[t][ct][0]);
            acc[t][ct][0] = mfma_f64(cim(a[t]), -bi, acc[t][ct][0]);
            acc[t][ct][1] = mfma_f64(cre(a[t]), bi, acc[t][ct][1]);
            acc[t][ct][1] = mfma_f64(cim(a[t]), br, acc[t][ct][1]);
          }
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[t][ct][0] = mfma_f64(cre(a[t]), br, acc[t][ct][0]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const int j = ct * 16 + i16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = row0 + t * 16 + 4 * v + q;
          if (r < n && j < kc) {
            A out;
            if constexpr (CPX) out = A{acc[t][ct][0][v], acc[t][ct][1][v]};
            else out = acc[t][ct][0][v];
            C[(int64_t)j * ldc + r] = narrow<T>(out);
          }
        }
      }
  }
}

// LDS of the matrix-core product for l0 basis columns (0: too many for it).
template <class T>
static size_t gemm_mfma_lds(int l0, int nct) {
  const size_t bytes = (size_t)((l0 + 3) & ~3) * 16 * nct * sizeof(double) * (traits<T>::cpx ? 2 : 1);
  return bytes <= 144 * 1024 ? bytes : 0;
}

// Columns of R^{-1} (R: n x n upper triangular, ld ldr), a wave per column
// j: x = e_j, then for i = j down to 0: x_i /= R(i, i) and x(0:i) -= x_i
// R(0:i, i), lane l holding rows l + 64 q (q < kTriRows); column i + 1 of R
// is loaded while column i is applied.  Writes Ri(:, j) (ld ldri, zeros below
// j) and ||Ri(:, j)||^2 to fro2[j].  n <= 64 kTriRows.
constexpr int kTriRows = 8;
template <class A>
__global__ __launch_bounds__(64) void k_tri_inv_cols(int n, const A* __restrict__ R, int ldr, A* __restrict__ Ri,
                                                     int ldri, double* __restrict__ fro2) {
  const int j = blockIdx.x, lane = threadIdx.x;
  A x[kTriRows];
#pragma unroll
  for (int q = 0; q < kTriRows; ++q) {
    A v = zero<A>();
    if (lane + 64 * q == j) *(double*)&v = 1.0;
    x[q] = v;
  }
  A col[kTriRows], nxt[kTriRows];
  auto load = [&](int i, A (&c)[kTriRows]) {
#pragma unroll
    for (int q = 0; q < kTriRows; ++q) {
      const int r = lane + 64 * q;
      c[q] = r <= i && r < n ? R[(int64_t)i * ldr + r] : zero<A>();
    }
  };
  load(j, nxt);
  for (int i = j; i >= 0; --i) {
#pragma unroll
    for (int q = 0; q < kTriRows; ++q) col[q] = nxt[q];
    if (i > 0) load(i - 1, nxt);
    // x_i /= R(i, i): the owner lane's entry, broadcast
    const int ow = i & 63, oq = i >> 6;
    A xi = zero<A>(), rii = zero<A>();
#pragma unroll
    for (int q = 0; q < kTriRows; ++q)
      if (q == oq) {
        xi = x[q];
        rii = col[q];
      }
    xi = shfl_v(xi, ow);
    rii = shfl_v(rii, ow);
    const double d = abs2(rii);
    xi = d > 0.0 ? scale(xi * conj(rii), 1.0 / d) : zero<A>();
#pragma unroll
    for (int q = 0; q < kTriRows; ++q) {
      const int r = lane + 64 * q;
      if (r == i) x[q] = xi;
      else if (r < i) x[q] -= col[q] * xi;
    }
  }
  double nr = 0.0;
#pragma unroll
  for (int q = 0; q < kTriRows; ++q) {
    const int r = lane + 64 * q;
    if (r < n) {
      Ri[(int64_t)j * ldri + r] = r <= j ? x[q] : zero<A>();
      if (r <= j) nr += abs2(x[q]);
    }
  }
  nr = wave_sum(nr);
  if (lane == 0) fro2[j] = nr;
}

template <class A>
bool launch_tri_inverse(hipStream_t st, int n, const A* R, int ldr, A* Ri, int ldri, double* fro2) {
  if (n < 1 || n > 64 * kTriRows) return false;
  hipLaunchKernelGGL(k_tri_inv_cols<A>, dim3(n), dim3(64), 0, st, n, R, ldr, Ri, ldri, fro2);
  return true;
}

int gemm_basis_width(int kc) { return kc <= 8 ? 8 : (kc + 7) / 8 * 8; }

template <class T>
void launch_gemm_basis(hipStream_t st, int n, const T* U, int64_t ldu, int ku, const T* P,
                       int64_t ldp, int jp, const typename traits<T>::acc* G, int kc, T* C,
                       int64_t ldc) {
  const int nb = (n + kBlock - 1) / kBlock;
  const int ldg = gemm_basis_width(kc);
  // complex data on the matrix cores (real data streams faster through the
  // vector kernel below), output columns in launches of at most 32
  if (traits<T>::cpx && gemm_mfma_lds<T>(ku + jp, 2) > 0) {
    static int ncu[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (ncu[dev] == 0 && hipDeviceGetAttribute(&ncu[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu[dev] = 256;
    // one workgroup per CU (its LDS), 32 CUs left free: the product runs
    // beside the least squares, whose small launches would otherwise wait for
    // it to drain
    const int blocks = (n + kGemmMfmaRows - 1) / kGemmMfmaRows;
    const int grid = std::max(1, std::min(blocks, ncu[dev] >= 128 ? ncu[dev] - 32 : ncu[dev]));
    for (int c0 = 0; c0 < kc; c0 += 32) {
      const int cc = std::min(32, kc - c0);
      const int nct = cc <= 16 ? 1 : 2;
      const size_t lds = gemm_mfma_lds<T>(ku + jp, nct);
      if (nct == 1)
        hipLaunchKernelGGL((k_gemm_basis_mfma<T, 1>), dim3(grid), dim3(kGemmMfmaThreads), lds, st, n, U, ldu, ku,
                           P, ldp, jp, G + c0, ldg, cc, C + (int64_t)c0 * ldc, ldc);
      else
        hipLaunchKernelGGL((k_gemm_basis_mfma<T, 2>), dim3(grid), dim3(kGemmMfmaThreads), lds, st, n, U, ldu, ku,
                           P, ldp, jp, G + c0, ldg, cc, C + (int64_t)c0 * ldc, ldc);
    }
    return;
  }
  // real data, even sizes and two-element aligned columns: two rows per
  // thread while the accumulators fit (output columns in launches of at most
  // 24)
  if constexpr (!traits<T>::cpx) {
    auto even2 = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % (2 * sizeof(T)) == 0; };
    if (n % 2 == 0 && ldu % 2 == 0 && ldp % 2 == 0 && ldc % 2 == 0 && even2(U) && even2(P) && even2(C)) {
      const int nb2 = (n / 2 + kBlock - 1) / kBlock;
      for (int c0 = 0; c0 < kc; c0 += 24) {
        const int cc = std::min(24, kc - c0);
        const auto* Gc = G + c0;
        T* Cc = C + (int64_t)c0 * ldc;
        if (cc <= 8)
          hipLaunchKernelGGL((k_gemm_basis2<T, 8>), dim3(nb2), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp, jp,
                             Gc, ldg, cc, Cc, ldc);
        else if (cc <= 16)
          hipLaunchKernelGGL((k_gemm_basis2<T, 16>), dim3(nb2), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp,
                             jp, Gc, ldg, cc, Cc, ldc);
        else if (cc <= 20)
          hipLaunchKernelGGL((k_gemm_basis2<T, 20>), dim3(nb2), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp,
                             jp, Gc, ldg, cc, Cc, ldc);
        else
          hipLaunchKernelGGL((k_gemm_basis2<T, 24>), dim3(nb2), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp,
                             jp, Gc, ldg, cc, Cc, ldc);
      }
      return;
    }
  }
  // output columns in launches of at most 32 (the padded row width covers
  // the last one)
  for (int c0 = 0; c0 < kc; c0 += 32) {
    const int km = gemm_basis_width(kc - c0 < 32 ? kc - c0 : 32);
    const int cc = kc - c0 < km ? kc - c0 : km;
    const auto* Gc = G + c0;
    T* Cc = C + (int64_t)c0 * ldc;
    if (km == 8)
      hipLaunchKernelGGL((k_gemm_basis<T, 8>), dim3(nb), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp, jp,
                         Gc, ldg, cc, Cc, ldc);
    else if (km == 16)
      hipLaunchKernelGGL((k_gemm_basis<T, 16>), dim3(nb), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp,
                         jp, Gc, ldg, cc, Cc, ldc);
    else if (km == 24 && cc <= 20)  // (k = 20: no multiply-adds on padding columns)
      hipLaunchKernelGGL((k_gemm_basis<T, 20>), dim3(nb), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp,
                         jp, Gc, ldg, cc, Cc, ldc);
    else if (km == 24)
      hipLaunchKernelGGL((k_gemm_basis<T, 24>), dim3(nb), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp,
                         jp, Gc, ldg, cc, Cc, ldc);
    else
      hipLaunchKernelGGL((k_gemm_basis<T, 32>), dim3(nb), dim3(kBlock), 0, st, n, U, ldu, ku, P, ldp,
                         jp, Gc, ldg, cc, Cc, ldc);
  }
}

// Small dense products of the least squares and the eigen-step (M, N up to a
// few hundred, K up to the sketch size).
// C = A^H B: one wave per entry of C, a dot product of two columns of length
// K with the lanes over K (coalesced), then a fixed-order wave sum.
template <class A>
__global__ __launch_bounds__(kBlock) void k_small_gemm_ct(int M, int N, int K, const A* __restrict__ a, int lda,
                                                          const A* __restrict__ b, int ldb, A* __restrict__ c,
                                                          int ldc) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (o >= M * N) return;  // the whole wave leaves together
  const int i = o % M, jc = o / M;
  const A* ai = a + (int64_t)i * lda;
  const A* bj = b + (int64_t)jc * ldb;
  A sum = zero<A>();
  for (int k = lane; k < K; k += 64) sum += conj(ai[k]) * bj[k];
  sum = wave_sum(sum);
  if (lane == 0) c[(int64_t)jc * ldc + i] = sum;
}

// C = A B: a block per 64 rows of one column of C, the lanes over the rows
// (coalesced loads of A), the K terms split over the block's waves (eight
// loads in flight per round) and the wave partials added in a fixed order.
template <class A>
__global__ __launch_bounds__(kBlock) void k_small_gemm_nn(int M, int N, int K, const A* __restrict__ a, int lda,
                                                          const A* __restrict__ b, int ldb, A* __restrict__ c,
                                                          int ldc) {
  __shared__ A part[kWaves * 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane, jc = blockIdx.y;
  const int kc = (K + kWaves - 1) / kWaves, k0 = wv * kc, k1 = min(K, k0 + kc);
  const int ic = min(i, M - 1);
  const A* bj = b + (int64_t)jc * ldb;
  A sum = zero<A>();
  int k = k0;
  for (; k + 8 <= k1; k += 8) {
    A v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = a[(int64_t)(k + u) * lda + ic];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += v[u] * bj[k + u];
  }
  for (; k < k1; ++k) sum += a[(int64_t)k * lda + ic] * bj[k];
  part[wv * 64 + lane] = sum;
  __syncthreads();
  if (wv == 0 && i < M) {
    A t = part[lane];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) t += part[w * 64 + lane];
    c[(int64_t)jc * ldc + i] = t;
  }
}

template <class A>
void launch_small_gemm(hipStream_t st, bool ct, int M, int N, int K, const A* a, int lda,
                       const A* b, int ldb, A* c, int ldc) {
  if (M * N == 0) return;
  if (ct) {
    const int nb = (M * N + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(k_small_gemm_ct<A>, dim3(nb), dim3(kBlock), 0, st, M, N, K, a, lda, b, ldb, c, ldc);
  } else {
    hipLaunchKernelGGL(k_small_gemm_nn<A>, dim3((M + 63) / 64, N), dim3(kBlock), 0, st, M, N, K, a, lda, b,
                       ldb, c, ldc);
  }
}

// ------------------------------------------------- triangular solve --
__device__ __forceinline__ bool nonzero(double v) { return v != 0.0; }
__device__ __forceinline__ bool nonzero(cx<double> v) { return v.x != 0.0 || v.y != 0.0; }
__device__ __forceinline__ double div(double a, double b) { return a / b; }
__device__ __forceinline__ cx<double> div(cx<double> a, cx<double> b) {
  const double d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__device__ __forceinline__ cx<double> read_lane(cx<double> v, int l) { return {read_lane(v.x, l), read_lane(v.y, l)}; }

// y = R^{-1} z over the leading nls columns of the upper triangular R (ld
// ldr), then the coefficients of the stored basis: y_i for the recycled
// columns (i < khat) and y_i / nu_{i-khat} for the unnormalised P columns.
// One wave; lane l owns rows l + 64 q (q < RPL).  Column entries are loaded
// eight columns ahead; y_i is broadcast from its owner lane and every row
// k < i subtracts R(k, i) y_i, in the order of a sequential back substitution.
template <class A, int RPL>
__global__ __launch_bounds__(64) void k_back_subst(int nls, int khat, const A* __restrict__ R, int ldr,
                                                   const A* __restrict__ z, const double* __restrict__ nu,
                                                   A* __restrict__ yout) {
  const int lane = threadIdx.x;
  A y[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int k = lane + 64 * q;
    y[q] = k < nls ? z[k] : zero<A>();
  }
  for (int i = nls - 1; i >= 0; i -= 8) {
    A rc[8][RPL], rd[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = max(i - u, 0);
      const A* col = R + (int64_t)c * ldr;
#pragma unroll
      for (int q = 0; q < RPL; ++q) rc[u][q] = col[min(lane + 64 * q, ldr - 1)];
      rd[u] = col[c];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = i - u;
      if (c >= 0) {
        A yc = zero<A>();
#pragma unroll
        for (int q = 0; q < RPL; ++q)
          if (q == c / 64) yc = read_lane(y[q], c & 63);
        yc = nonzero(rd[u]) ? div(yc, rd[u]) : zero<A>();
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          const int k = lane + 64 * q;
          if (k == c) y[q] = yc;
          else if (k < c) y[q] -= rc[u][q] * yc;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int k = lane + 64 * q;
    if (k < nls) yout[k] = k < khat ? y[q] : scale(y[q], 1.0 / nu[k - khat]);
  }
}

template <class A>
bool launch_back_subst(hipStream_t st, int nls, int khat, const A* R, int ldr, const A* z, const double* nu,
                       A* y) {
  if (nls <= 0) return true;
  if (nls <= 128)
    hipLaunchKernelGGL((k_back_subst<A, 2>), dim3(1), dim3(64), 0, st, nls, khat, R, ldr, z, nu, y);
  else if (nls <= 256)
    hipLaunchKernelGGL((k_back_subst<A, 4>), dim3(1), dim3(64), 0, st, nls, khat, R, ldr, z, nu, y);
  else if (nls <= 512)
    hipLaunchKernelGGL((k_back_subst<A, 8>), dim3(1), dim3(64), 0, st, nls, khat, R, ldr, z, nu, y);
  else
    return false;
  return true;
}

// ------------------------------------------------------------ elementwise --
template <class A>
__global__ void k_axpy(int n, A alpha, const A* __restrict__ x, A* __restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    y[i] += alpha * x[i];
}
template <class A> void launch_axpy(hipStream_t st, int n, A alpha, const A* x, A* y) {
  hipLaunchKernelGGL(k_axpy<A>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n, alpha, x, y);
}

// A cycle's control block, cleared by the launch that forms its first basis
// vector (one launch fewer at each cycle start).
__device__ __forceinline__ void set_ctrl_fields(Ctrl* c, double thresh) {
  c->halt = 0;
  c->halt_j = 0;
  c->flags = 0;
  c->thresh = thresh;
}

template <class T>
__global__ void k_cast_scale(int n, const typename traits<T>::acc* __restrict__ src, double s,
                             T* __restrict__ dst, Ctrl* ctrl, double thresh) {
  if (ctrl && blockIdx.x == 0 && threadIdx.x == 0) set_ctrl_fields(ctrl, thresh);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = narrow<T>(scale(src[i], s));
}
template <class T>
void launch_cast_scale(hipStream_t st, int n, const typename traits<T>::acc* src, double s, T* dst,
                       Ctrl* ctrl, double thresh) {
  hipLaunchKernelGGL(k_cast_scale<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n, src,
                     s, dst, ctrl, thresh);
}

template <class T>
__global__ void k_cast_rscale(int n, const typename traits<T>::acc* __restrict__ src,
                              const typename traits<T>::acc* __restrict__ nrm2, T* __restrict__ dst,
                              Ctrl* ctrl, double thresh) {
  if (ctrl && blockIdx.x == 0 && threadIdx.x == 0) set_ctrl_fields(ctrl, thresh);
  const double q = re(nrm2[0]);
  const double sc = q > 0.0 ? 1.0 / sqrt(q) : 1.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = narrow<T>(scale(src[i], sc));
}
template <class T>
void launch_cast_rscale(hipStream_t st, int n, const typename traits<T>::acc* src,
                        const typename traits<T>::acc* nrm2, T* dst, Ctrl* ctrl, double thresh) {
  hipLaunchKernelGGL(k_cast_rscale<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n, src, nrm2,
                     dst, ctrl, thresh);
}

template <class T>
__global__ void k_widen_scale(int n, const T* __restrict__ src, double s,
                              typename traits<T>::acc* __restrict__ dst) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = scale(widen(src[i]), s);
}
template <class T>
void launch_widen_scale(hipStream_t st, int n, const T* src, double s, typename traits<T>::acc* dst) {
  hipLaunchKernelGGL(k_widen_scale<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n, src,
                     s, dst);
}

template <class T>
__global__ void k_narrow_values(int64_t n, const typename traits<T>::acc* __restrict__ src,
                                T* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = narrow<T>(src[i]);
}
template <class T>
void launch_narrow_values(hipStream_t st, int64_t n, const typename traits<T>::acc* src, T* dst) {
  const int nb = (int)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_narrow_values<T>, dim3(nb), dim3(kBlock), 0, st, n, src, dst);
}

template <class A>
__global__ void k_gather_conj(int64_t nnz, const A* __restrict__ src, const int* __restrict__ perm,
                              A* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = conj(src[perm[i]]);
}
template <class A>
void launch_gather_conj(hipStream_t st, int64_t nnz, const A* src, const int* perm, A* dst) {
  const int nb = (int)((nnz + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_gather_conj<A>, dim3(nb), dim3(kBlock), 0, st, nnz, src, perm, dst);
}

template <class A>
__global__ void k_grad_values(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                              const A* __restrict__ lam, const A* __restrict__ x, A* __restrict__ g) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const A l = lam[r];
    const int e1 = rp[r + 1];
    for (int e = rp[r]; e < e1; ++e) g[e] = -(l * conj(x[ci[e]]));
  }
}
template <class A>
void launch_grad_values(hipStream_t st, int n, const int* rp, const int* ci, const A* lam,
                        const A* x, A* g) {
  hipLaunchKernelGGL(k_grad_values<A>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n, rp,
                     ci, lam, x, g);
}

__global__ void k_set_ctrl(Ctrl* c, int halt, double thresh) {
  if (threadIdx.x == 0) {
    c->halt = halt;
    c->halt_j = 0;
    c->flags = 0;
    c->thresh = thresh;
  }
}
void launch_set_ctrl(hipStream_t st, Ctrl* c, int halt, double thresh) {
  hipLaunchKernelGGL(k_set_ctrl, dim3(1), dim3(64), 0, st, c, halt, thresh);
}

__global__ void k_set_ctrl_givens(Ctrl* c, double thresh, double eps, double est, double sprev) {
  if (threadIdx.x == 0) {
    c->halt = 0;
    c->halt_j = 0;
    c->flags = 0;
    c->thresh = thresh;
    c->eps = eps;
    c->est = est;
    c->sprev = sprev;
  }
}
void launch_set_ctrl_givens(hipStream_t st, Ctrl* c, double thresh, double eps, double est, double sprev) {
  hipLaunchKernelGGL(k_set_ctrl_givens, dim3(1), dim3(64), 0, st, c, thresh, eps, est, sprev);
}

// ------------------------------------------- right Jacobi preconditioning ---
// A D^-1 with D = diag(A): d from each row's stored diagonal entry (zero if
// the row stores none, which sets *flag), the column-scaled values
// a_ij * (1 / d_j), and x <- x * d or x * (1 / d) for the change of variable
// x = D^-1 u.
__device__ __forceinline__ double recip(double d) { return 1.0 / d; }
__device__ __forceinline__ cx<double> recip(cx<double> d) { return scale(conj(d), 1.0 / abs2(d)); }

template <class A>
__global__ void k_jacobi_diag(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                              const A* __restrict__ val, A* __restrict__ d, int* __restrict__ flag) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    A v = zero<A>();
    const int e1 = rp[r + 1];
    for (int e = rp[r]; e < e1; ++e)
      if (ci[e] == r) v = val[e];
    d[r] = v;
    if (abs2(v) == 0.0) flag[0] = 1;
  }
}

template <class A>
__global__ void k_scale_cols(int64_t nnz, const int* __restrict__ ci, const A* __restrict__ val,
                             const A* __restrict__ d, A* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = val[e] * recip(d[ci[e]]);
}

template <class A>
void launch_jacobi(hipStream_t st, int n, int64_t nnz, const int* rp, const int* ci, const A* val, A* d,
                   A* scaled, int* flag) {
  hipLaunchKernelGGL(k_jacobi_diag<A>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n, rp, ci, val, d,
                     flag);
  if (nnz > 0) {
    const int64_t nb = std::min<int64_t>((nnz + kBlock - 1) / kBlock, 1 << 20);
    hipLaunchKernelGGL(k_scale_cols<A>, dim3((unsigned)nb), dim3(kBlock), 0, st, nnz, ci, val, d, scaled);
  }
}

template <class A>
__global__ void k_scale_by_diag(int n, const A* __restrict__ d, A* __restrict__ x, int divide) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    x[i] = x[i] * (divide ? recip(d[i]) : d[i]);
}

template <class A>
void launch_scale_by_diag(hipStream_t st, int n, const A* d, A* x, bool divide) {
  hipLaunchKernelGGL(k_scale_by_diag<A>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n, d, x,
                     divide ? 1 : 0);
}

// ------------------------------------------------------------- ILU(0) ---
// One thread per row of the colour being eliminated: the row's entries left
// of the diagonal in elimination order, in that order, each divided by its
// pivot (a row of an earlier colour, already final) and its updates applied
// to the row's own entries.
template <class A>
__global__ void k_ilu_factor(int cnt, const int* __restrict__ rows, const int* __restrict__ lo_off,
                             const int2* __restrict__ lo, const int* __restrict__ up_off,
                             const int2* __restrict__ up, const int* __restrict__ dpos, A* __restrict__ F,
                             int* __restrict__ flag) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += gridDim.x * blockDim.x) {
    const int i = rows[t];
    for (int l = lo_off[i]; l < lo_off[i + 1]; ++l) {
      const int2 pk = lo[l];
      const A lik = F[pk.x] * recip(F[pk.y]);
      F[pk.x] = lik;
      for (int u = up_off[l]; u < up_off[l + 1]; ++u) {
        const int2 q = up[u];
        F[q.x] -= lik * F[q.y];
      }
    }
    if (abs2(F[dpos[i]]) == 0.0) flag[0] = 1;
  }
}

// Forward solve of one colour from its packed lower entries: y_i = in_i -
// sum of l_ik y_k (the k of earlier colours; src is y, or in itself when
// every earlier row is of colour 0, where y = in).  For the last colour also
// the backward step z_i = y_i / u_ii (no entries right of its diagonal);
// y is then not stored unless asked for.
template <class T>
__global__ void k_ilu_fwd(int cnt, const int* __restrict__ rows, const int* __restrict__ sl_off,
                          const int* __restrict__ sl_w, const int* __restrict__ col,
                          const typename traits<T>::acc* __restrict__ val,
                          const typename traits<T>::acc* __restrict__ dinv, const T* __restrict__ in,
                          const typename traits<T>::acc* __restrict__ ysrc, int src_in,
                          typename traits<T>::acc* __restrict__ y, T* __restrict__ z, int last,
                          const Ctrl* __restrict__ ctrl) {
  using A = typename traits<T>::acc;
  if (ctrl && ctrl->halt) return;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += gridDim.x * blockDim.x) {
    const int sl = t >> 6, lane = t & 63;
    const int i = rows[t];
    A acc = widen(in[i]);
    const int o = sl_off[sl], w = sl_w[sl];
    for (int k = 0; k < w; ++k) {
      const int c = col[o + k * 64 + lane];
      const A v = val[o + k * 64 + lane];
      acc -= v * (src_in ? widen(in[c]) : ysrc[c]);
    }
    if (y) y[i] = acc;
    if (last) z[i] = narrow<T>(acc * dinv[t]);
  }
}

// Backward solve of one colour from its packed upper entries: z_i = (y_i -
// sum of u_ij z_j) / u_ii, the j of later colours (y_i = in_i for colour 0).
template <class T>
__global__ void k_ilu_bwd(int cnt, const int* __restrict__ rows, const int* __restrict__ sl_off,
                          const int* __restrict__ sl_w, const int* __restrict__ col,
                          const typename traits<T>::acc* __restrict__ val,
                          const typename traits<T>::acc* __restrict__ dinv, const T* __restrict__ in,
                          const typename traits<T>::acc* __restrict__ y, T* __restrict__ z,
                          const Ctrl* __restrict__ ctrl) {
  using A = typename traits<T>::acc;
  if (ctrl && ctrl->halt) return;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += gridDim.x * blockDim.x) {
    const int sl = t >> 6, lane = t & 63;
    const int i = rows[t];
    A acc = y ? y[i] : widen(in[i]);
    const int o = sl_off[sl], w = sl_w[sl];
    for (int k = 0; k < w; ++k) {
      const int c = col[o + k * 64 + lane];
      const A v = val[o + k * 64 + lane];
      acc -= v * widen(z[c]);
    }
    z[i] = narrow<T>(acc * dinv[t]);
  }
}

// Packed factor copies: val[p] = F[src[p]] (0 for padding).
template <class A>
__global__ void k_ilu_pack(int64_t np, const int* __restrict__ src, const A* __restrict__ F, A* __restrict__ out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const int e = src[p];
    out[p] = e >= 0 ? F[e] : zero<A>();
  }
}

template <class A>
__global__ void k_ilu_dinv(int n, const int* __restrict__ rows, const int* __restrict__ dpos,
                           const A* __restrict__ F, A* __restrict__ dinv) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    dinv[t] = recip(F[dpos[rows[t]]]);
}

// t = U x over all rows (mode 0) or out = t + L t (mode 1).
template <class A>
__global__ void k_ilu_mult(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const uint8_t* __restrict__ kind, const A* __restrict__ F, const A* __restrict__ x,
                           A* __restrict__ out, int mode) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    A acc = mode == 0 ? zero<A>() : x[i];
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; ++e) {
      const int k = kind[e];
      if (mode == 0 ? k != 0 : k == 0) acc += F[e] * x[ci[e]];
    }
    out[i] = acc;
  }
}

static inline int ilu_grid(int cnt) { return std::max(1, std::min((cnt + kBlock - 1) / kBlock, 1 << 16)); }

template <class A>
void launch_ilu_factor(hipStream_t st, const IluView& v, const int* lo_off, const int2* lo, const int* up_off,
                       const int2* up, A* F, int* flag) {
  for (int c = 0; c < v.ncolours; ++c) {
    const int c0 = v.coff[c], cnt = v.coff[c + 1] - c0;
    if (cnt <= 0) continue;
    hipLaunchKernelGGL(k_ilu_factor<A>, dim3(ilu_grid(cnt)), dim3(kBlock), 0, st, cnt, v.crow + c0, lo_off, lo,
                       up_off, up, v.dpos, F, flag);
  }
}

// Colour 0 has no entries left of its diagonal (its rows neighbour no row of
// the same colour), so y = in there; with two colours the forward solve of
// colour 1 reads in directly and y is never stored: two launches.
template <class T>
void launch_ilu_apply(hipStream_t st, const IluView& v, const T* in, typename traits<T>::acc* y, T* out,
                      const Ctrl* ctrl) {
  using A = typename traits<T>::acc;
  const A* lval = static_cast<const A*>(v.lval);
  const A* uval = static_cast<const A*>(v.uval);
  const A* dinv = static_cast<const A*>(v.dinv);
  const int C = v.ncolours;
  const bool two = C <= 2;
  for (int c = 0; c < C; ++c) {
    const int c0 = v.coff[c], cnt = v.coff[c + 1] - c0;
    if (cnt <= 0) continue;
    if (c == 0 && C > 1 && two) continue;  // y = in for colour 0, read in place
    const int s0 = v.lsl0[c];
    hipLaunchKernelGGL(k_ilu_fwd<T>, dim3(ilu_grid(cnt)), dim3(kBlock), 0, st, cnt, v.crow + c0,
                       v.lslice + s0, v.lw + s0, v.lcol, lval, dinv + c0, in, (const A*)y, two ? 1 : 0,
                       two ? (A*)nullptr : y, out, c == C - 1 ? 1 : 0, ctrl);
  }
  for (int c = C - 2; c >= 0; --c) {
    const int c0 = v.coff[c], cnt = v.coff[c + 1] - c0;
    if (cnt <= 0) continue;
    const int s0 = v.usl0[c];
    hipLaunchKernelGGL(k_ilu_bwd<T>, dim3(ilu_grid(cnt)), dim3(kBlock), 0, st, cnt, v.crow + c0,
                       v.uslice + s0, v.uw + s0, v.ucol, uval, dinv + c0, in,
                       (c == 0 && two) ? (const A*)nullptr : (const A*)y, out, ctrl);
  }
}

template <class A>
void launch_ilu_pack(hipStream_t st, const IluView& v, int64_t nl, const int* lsrc, int64_t nu,
                     const int* usrc) {
  const A* F = static_cast<const A*>(v.F);
  auto grid = [](int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 1 << 16)); };
  if (nl > 0)
    hipLaunchKernelGGL(k_ilu_pack<A>, dim3(grid(nl)), dim3(kBlock), 0, st, nl, lsrc, F,
                       static_cast<A*>(const_cast<void*>(v.lval)));
  if (nu > 0)
    hipLaunchKernelGGL(k_ilu_pack<A>, dim3(grid(nu)), dim3(kBlock), 0, st, nu, usrc, F,
                       static_cast<A*>(const_cast<void*>(v.uval)));
  hipLaunchKernelGGL(k_ilu_dinv<A>, dim3(ilu_grid(v.n)), dim3(kBlock), 0, st, v.n, v.crow, v.dpos, F,
                     static_cast<A*>(const_cast<void*>(v.dinv)));
}

template <class A>
void launch_ilu_mult(hipStream_t st, const IluView& v, const A* x, A* t, A* out) {
  const A* F = static_cast<const A*>(v.F);
  hipLaunchKernelGGL(k_ilu_mult<A>, dim3(ilu_grid(v.n)), dim3(kBlock), 0, st, v.n, v.rp, v.ci, v.kind, F, x, t, 0);
  hipLaunchKernelGGL(k_ilu_mult<A>, dim3(ilu_grid(v.n)), dim3(kBlock), 0, st, v.n, v.rp, v.ci, v.kind, F, t, out,
                     1);
}

// ---------------------------------------------------- instantiations ---
#define SDR_INST_BASIS(T)                                                                        \
  template void launch_spmv_sketch<T>(hipStream_t, int, const int*, const int*, const T*,          \
                                      const T*, T*, Window<T>, int, SketchSpec, bool,             \
                                      traits<T>::acc*, int, const Ctrl*, hipEvent_t, hipEvent_t); \
  template void launch_spmv_dia_sketch<T>(hipStream_t, int, DiaView<T>, const T*, T*, Window<T>,  \
                                          int, SketchSpec, bool, traits<T>::acc*, int,           \
                                          const Ctrl*, hipEvent_t, hipEvent_t);                  \
  template void launch_pack_dia<T>(hipStream_t, int64_t, const traits<T>::acc*, const int*, T*);   \
  template void launch_dia_const<T>(hipStream_t, int, DiaView<T>, int*, T*);                       \
  template void launch_update<T>(hipStream_t, int, T*, Window<T>, int, const traits<T>::acc*, int, \
                                 int, double*, int, int, const Ctrl*, hipEvent_t, hipEvent_t);    \
  template void launch_sketch_cols<T>(hipStream_t, int, const T*, int64_t, int, SketchSpec,       \
                                      traits<T>::acc*, int);                                      \
  template void launch_dct_sketch<T>(hipStream_t, int, const T*, DctSpec, traits<T>::acc*, int, bool, \
                                     const Ctrl*, hipEvent_t, hipEvent_t);                        \
  template void launch_gemv_basis<T>(hipStream_t, int, const T*, int64_t, int, const T*, int64_t, \
                                     int, const traits<T>::acc*, traits<T>::acc*);                \
  template void launch_gemm_basis<T>(hipStream_t, int, const T*, int64_t, int, const T*, int64_t, \
                                     int, const traits<T>::acc*, int, T*, int64_t);               \
  template void launch_cast_scale<T>(hipStream_t, int, const traits<T>::acc*, double, T*, Ctrl*, double); \
  template void launch_cast_rscale<T>(hipStream_t, int, const traits<T>::acc*, const traits<T>::acc*, T*, \
                                       Ctrl*, double);                                             \
  template void launch_widen_scale<T>(hipStream_t, int, const T*, double, traits<T>::acc*);       \
  template void launch_narrow_values<T>(hipStream_t, int64_t, const traits<T>::acc*, T*);        \
  template void launch_ilu_apply<T>(hipStream_t, const IluView&, const T*, traits<T>::acc*, T*,    \
                                    const Ctrl*);

SDR_INST_BASIS(double)
SDR_INST_BASIS(float)
SDR_INST_BASIS(cx<double>)
SDR_INST_BASIS(cx<float>)

#define SDR_INST_ACC(A)                                                                         \
  template void launch_reduce_cols<A>(hipStream_t, const A*, int, int, int, double, A*,        \
                                      const Ctrl*, A*);                                         \
  template void launch_lsq_step<A>(hipStream_t, LsqState<A>, int, int, int, int, int, const A*, \
                                   double, double);                                             \
  template void launch_reduce2<A>(hipStream_t, const A*, int, int, int, double, const A*, int,  \
                                  int, A*, const Ctrl*);                                        \
  template void launch_init_v0<A>(hipStream_t, const A*, int, A*, double*);                     \
  template void launch_lsq_init<A>(hipStream_t, LsqState<A>, int, int, const A*, double, int, GivensInit, int); \
  template bool launch_tri_inverse<A>(hipStream_t, int, const A*, int, A*, int, double*);                    \
  template void launch_lsq_steps<A>(hipStream_t, LsqState<A>, int, int, int, int, int, int,      \
                                    const A*, int64_t, int, double, double, int);                \
  template void launch_reduce_steps<A>(hipStream_t, const A*, int64_t, int, int, int, int, int,  \
                                       int, double, A*, int64_t, const Ctrl*);                  \
  template void launch_backsolve<A>(hipStream_t, LsqState<A>, int, int, A*);                    \
  template void launch_spmv_dia_residual<A>(hipStream_t, int, DiaView<A>, const A*, const A*, A*, A*, \
                                            int, SketchSpec);                                       \
  template void launch_spmv_residual<A>(hipStream_t, int, const int*, const int*, const A*,     \
                                        const A*, const A*, A*, A*, int, SketchSpec);          \
  template bool launch_back_subst<A>(hipStream_t, int, int, const A*, int, const A*, const double*, A*); \
  template void launch_small_gemm<A>(hipStream_t, bool, int, int, int, const A*, int, const A*, \
                                     int, A*, int);                                             \
  template void launch_axpy<A>(hipStream_t, int, A, const A*, A*);                              \
  template void launch_jacobi<A>(hipStream_t, int, int64_t, const int*, const int*, const A*, A*, A*, \
                                 int*);                                                         \
  template void launch_scale_by_diag<A>(hipStream_t, int, const A*, A*, bool);                 \
  template void launch_gather_conj<A>(hipStream_t, int64_t, const A*, const int*, A*);          \
  template void launch_grad_values<A>(hipStream_t, int, const int*, const int*, const A*,       \
                                      const A*, A*);                                            \
  template void launch_ilu_factor<A>(hipStream_t, const IluView&, const int*, const int2*,      \
                                     const int*, const int2*, A*, int*);                        \
  template void launch_ilu_mult<A>(hipStream_t, const IluView&, const A*, A*, A*);               \
  template void launch_ilu_pack<A>(hipStream_t, const IluView&, int64_t, const int*, int64_t, const int*);

SDR_INST_ACC(double)
SDR_INST_ACC(cx<double>)

}  // namespace sdr
