// Diffusion kernels of the DAETI step B (paper Sec. 2): one forward-Euler
// substep of dt_ad on dV/dt = -M_L^-1 K V + s(tau), fused with the stimulus
// and written Jacobi-style (read Vin, write Vout), plus the FP64 Gershgorin
// bound of eq. (3) and a power iteration for lambda_max(M_L^-1 K).
//
// Both operator layouts use the difference form
//     V'_i = V_i + dt_ad * ( sum_{j != i} a_ij (V_j - V_i) + s_i ),
// with a_ij = -k_ij / m_i, which equals -(M_L^-1 K V)_i because every row
// of K sums to zero; a constant V is therefore reproduced exactly.
//
// Launch shape: one row per lane, 256 lanes per workgroup, 1-D grid.  The
// workgroup index is remapped so that each of the chip's 8 XCDs (which
// receive workgroups round-robin) works on one contiguous slice of rows: the
// neighbour rows a stencil reaches (up to one plane away) then stay in that
// XCD's L2.
#include <type_traits>

#include "grid_rows.h"
#include "mono_internal.h"

namespace mono {

// Workgroup index of this block.  With `remap`, logical blocks are dealt so
// that XCD x (which receives hardware workgroups x, x+8, x+16, ...) owns one
// contiguous range of rows.
__device__ __forceinline__ int64_t row_block(int64_t nb, int remap) {
  const int64_t b = blockIdx.x;
  if (!remap) return b;
  const int64_t x = b & 7, idx = b >> 3;
  const int64_t per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + idx;
}

// R consecutive values starting at an R-aligned index, in one vector access
template <int R, typename T>
__device__ __forceinline__ void vload(const T* p, T (&v)[R]) {
  if constexpr (R == 1) {
    v[0] = p[0];
  } else if constexpr (R == 2 && sizeof(T) == 4) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    v[0] = t.x; v[1] = t.y;
  } else if constexpr (R == 4 && sizeof(T) == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  } else if constexpr (R == 2 && sizeof(T) == 8) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    v[0] = t.x; v[1] = t.y;
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = p[r];
  }
}
template <int R, typename T>
__device__ __forceinline__ void vstore(T* p, const T (&v)[R]) {
  if constexpr (R == 1) {
    p[0] = v[0];
  } else if constexpr (R == 2 && sizeof(T) == 4) {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  } else if constexpr (R == 4 && sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 2 && sizeof(T) == 8) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) p[r] = v[r];
  }
}

__device__ __forceinline__ double tmul(double a, double b) { return rn_mul(a, b); }
__device__ __forceinline__ double tadd(double a, double b) { return rn_add(a, b); }

// Start time of this substep, evaluated exactly as t_n (+ dt/2) + m dt_ad
// with one rounding per operation (no contraction), so that stimulus windows
// open and close on the same substeps on every implementation.
__device__ __forceinline__ double substep_time(const StepClock& c, int half, int m,
                                               double dt_ad) {
  const int64_t step = *c.base + c.g;
  double t0 = tmul((double)step, c.dt);
  if (half) t0 = tadd(t0, tmul(0.5, c.dt));
  return tadd(t0, tmul((double)m, dt_ad));
}

template <typename T>
__device__ __forceinline__ T stimulus_rate(const DiffArgs<T>& a, int64_t i, double tau) {
  if (a.stim.n == 0 || a.stim_mask == nullptr) return T(0);
  uint32_t active = 0;
  for (int s = 0; s < a.stim.n; ++s)
    if (a.stim.t_on[s] <= tau && tau < a.stim.t_end[s]) active |= 1u << s;
  if (!active) return T(0);
  const uint32_t mask = a.stim_mask[i] & active;
  T r = T(0);
  for (int s = 0; s < a.stim.n; ++s)
    if (mask & (1u << s)) r += (T)a.stim.amp[s];
  return r;
}

// Stimuli open on this substep of a single instance (bit s for stimulus s):
// by the integer substep windows when the table carries them (no floating
// point on the way), else from the start time tau.
template <typename T>
__device__ __forceinline__ uint32_t open_stimuli(const DiffArgs<T>& a, double dt_ad) {
  if (a.stim.n == 0 || a.stim_mask == nullptr) return 0u;
  uint32_t active = 0;
  if (a.stim.L > 0) {
    const int64_t q = ((*a.clk.base + a.clk.g) * 2 + a.half) * (int64_t)a.stim.L + a.m;
    for (int s = 0; s < a.stim.n; ++s)
      if (a.stim.q_on[s] <= q && q < a.stim.q_end[s]) active |= 1u << s;
  } else {
    const double tau = substep_time(a.clk, a.half, a.m, dt_ad);
    for (int s = 0; s < a.stim.n; ++s)
      if (a.stim.t_on[s] <= tau && tau < a.stim.t_end[s]) active |= 1u << s;
  }
  return active;
}
// The same for substep m of this launch's half step.
template <typename T>
__device__ __forceinline__ uint32_t open_stimuli_at(const DiffArgs<T>& a, double dt_ad, int m) {
  DiffArgs<T> b = a;
  b.m = m;
  return open_stimuli(b, dt_ad);
}
// summed amplitude of the open stimuli that include node i
template <typename T>
__device__ __forceinline__ T stimulus_sum(const DiffArgs<T>& a, uint32_t active, int64_t i) {
  const uint32_t mask = a.stim_mask[i] & active;
  T r = T(0);
  for (int s = 0; s < a.stim.n; ++s)
    if (mask & (1u << s)) r += (T)a.stim.amp[s];
  return r;
}

// WC > 0: the ELL width as a compile-time constant (the slot loop unrolls,
// so every slot's column and value loads, then every gather, are in flight
// together); WC = 0 reads it at run time.  Same sums in the same order.
template <typename T, bool BATCHED, int BLOCK, int WC>
__global__ __launch_bounds__(BLOCK) void k_diff_ell(DiffArgs<T> a) {
  const int64_t nb = (a.n + BLOCK - 1) / BLOCK;
  const int64_t i = row_block(nb, a.xcd) * BLOCK + threadIdx.x;
  if (i >= a.n) return;
  const int q = BATCHED ? a.inst[i] : 0;
  const T vi = a.Vin[i];
  if (BATCHED && a.m >= a.l[q]) {   // this instance has finished its substeps
    a.Vout[i] = vi;
    return;
  }
  const double dt_ad = a.dt_ad[q];
  T acc = T(0);
  if constexpr (WC > 0) {
    int32_t j[WC];
    T v[WC];
#pragma unroll
    for (int s = 0; s < WC; ++s) {
      const int64_t k = (int64_t)s * a.Np + i;
      j[s] = a.col[k];
      v[s] = a.val[k];
    }
#pragma unroll
    for (int s = 0; s < WC; ++s) acc += v[s] * (a.Vin[j[s]] - vi);
  } else {
    for (int s = 0; s < a.W; ++s) {
      const int64_t k = (int64_t)s * a.Np + i;
      const int32_t j = a.col[k];
      acc += a.val[k] * (a.Vin[j] - vi);
    }
  }
  const double tau = substep_time(a.clk, a.half, a.m, dt_ad);
  acc += stimulus_rate(a, i, tau);
  a.Vout[i] = vi + (T)dt_ad * acc;
}

// Symmetric stencil: e[p][i] = -k(i, i+off_p) stored once per edge; row i
// gathers its forward edges from e[p][i] and its backward edges from
// e[p][i-off_p] (the edge stored by the neighbour).  Within an instance the
// entries of absent neighbours are zero, so clamping only keeps loads in
// bounds; a backward neighbour before the instance's first node belongs to
// another instance (whose slots mean other offsets) and is skipped.
// Each lane owns RPL consecutive rows: its own edges, 1/m, V_i and the result
// move as RPL-wide vector accesses; the neighbour gathers stay scalar.
// P = 0 reads the number of offsets at run time.  Padding rows (n <= i < Np)
// have zero edges, zero 1/m and zero potential, so they are computed as 0.
// NARROW: every row index and byte offset within one row array fits 32 bits
// (Np * sizeof(T) < 2^31), so indices are 32-bit and the loads take a
// uniform base plus a 32-bit offset (no 64-bit address arithmetic per
// neighbour).  Same loads, clamps and sums either way.
template <typename T, int P, bool BATCHED, int BLOCK, int RPL, bool NARROW>
__global__ __launch_bounds__(BLOCK) void k_diff_stencil(DiffArgs<T> a) {
  using I = typename std::conditional<NARROW, int, int64_t>::type;
  const int64_t nlanes = (a.n + RPL - 1) / RPL;
  const int64_t nb = (nlanes + BLOCK - 1) / BLOCK;
  const int64_t lane = row_block(nb, a.xcd) * BLOCK + threadIdx.x;
  if (lane * RPL >= a.n) return;
  const I i0 = (I)(lane * RPL);
  const int np = P > 0 ? P : a.P;
  const I last = (I)(a.n - 1);
  auto ld = [](const T* base, I j) -> T {
    if constexpr (NARROW)
      return ld_bytes(base, (uint32_t)j * (uint32_t)sizeof(T));
    else
      return base[j];
  };
  T vi[RPL], acc[RPL];
  vload<RPL>(a.Vin + i0, vi);
  int q[RPL];
  I first[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    q[r] = BATCHED ? a.inst[i0 + r] : 0;
    first[r] = BATCHED ? (I)a.inst_off[q[r]] : I(0);
    acc[r] = T(0);
  }
  auto edge = [&](int p) {
    const T* ep = a.e + (int64_t)p * a.Np;
    T wf[RPL];
    vload<RPL>(ep + i0, wf);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const I i = i0 + r;
      const I o = (I)a.off[q[r] * np + p];
      const I jf = i + o;
      const I jb = i - o;
      const I jbc = jb >= first[r] ? jb : first[r];
      // loaded unconditionally (jbc is always a row of this instance), so
      // that no branch holds the slots' loads apart
      const T wbl = ld(ep, jbc);
      const T wb = (jb >= first[r]) ? wbl : T(0);
      const T vf = ld(a.Vin, jf <= last ? jf : last);
      const T vb = ld(a.Vin, jbc);
      acc[r] += wf[r] * (vf - vi[r]);
      acc[r] += wb * (vb - vi[r]);
    }
  };
  if constexpr (P > 0) {
#pragma unroll
    for (int p = 0; p < P; ++p) edge(p);
  } else {
    for (int p = 0; p < np; ++p) edge(p);
  }
  T mv[RPL], out[RPL];
  vload<RPL>(a.minv + i0, mv);
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int64_t i = (int64_t)i0 + r;
    if (BATCHED && a.m >= a.l[q[r]]) {
      out[r] = vi[r];
      continue;
    }
    const double dt_ad = a.dt_ad[q[r]];
    const double tau = substep_time(a.clk, a.half, a.m, dt_ad);
    const T sr = (i < a.n) ? stimulus_rate(a, i, tau) : T(0);
    out[r] = vi[r] + (T)dt_ad * (mv[r] * acc[r] + sr);
  }
  vstore<RPL>(a.Vout + i0, out);
}

// The stencil sweep of a single instance whose rows are stored by class:
// row i reads only V, its class id and (through the class) a table row that
// the rows of a wavefront usually share, so HBM carries V in, V out and 2
// bytes per row.  Where every lane of a wavefront has the same class the
// table row is read through scalar loads.  Same arithmetic, in the same order,
// as k_diff_stencil with RPL = 1.

// Workgroup w sweeps ITER chunks of BLOCK consecutive rows, so the uniform
// work of a wavefront (arguments, substep time, open stimulus windows) is paid
// once per ITER rows.
template <typename T, int P, int BLOCK, int ITER>
__global__ __launch_bounds__(BLOCK) void k_diff_classes(DiffArgs<T> a) {
  constexpr int ES = (int)sizeof(T);
  const int64_t nb = (a.n + (int64_t)BLOCK * ITER - 1) / ((int64_t)BLOCK * ITER);
  const int64_t r0 = row_block(nb, a.xcd) * BLOCK * ITER;
  const int np = P > 0 ? P : a.P;
  const int n = (int)a.n;
  const int blast = (n - 1) * ES;
  const int maxo = a.off[np - 1];
  const T* V = a.Vin;
  const double dt_ad = a.dt_ad[0];
  const T hT = (T)dt_ad;
  const uint32_t active = open_stimuli(a, dt_ad);
  using Clamp = std::integral_constant<bool, true>;
  using NoClamp = std::integral_constant<bool, false>;
  for (int it = 0; it < ITER; ++it) {
    // rows addressed by 32-bit byte offsets from uniform bases (the host
    // takes this kernel only when n * sizeof(T) < 2^31)
    const int i = (int)(r0 + it * BLOCK) + (int)threadIdx.x;
    if (i >= n) break;
    const int bi = i * ES;
    const T vi = ld_bytes(V, (uint32_t)bi);
    const int c = a.cls[(uint32_t)i];
    const int c0 = __builtin_amdgcn_readfirstlane(c);
    // a wavefront whose rows all have every neighbour in range skips the clamps
    const bool inner = __ballot(i < maxo || i > n - 1 - maxo) == 0ull;
    T acc = T(0), mv;
    auto sweep = [&](const T* w, auto clamp) {
      auto edge = [&](int p) {
        const int bo = a.off[p] * ES;
        int bf = bi + bo, bb = bi - bo;
        if constexpr (decltype(clamp)::value) {
          bf = min(bf, blast);
          bb = max(bb, 0);
        }
        const T vf = ld_bytes(V, (uint32_t)bf);
        const T vb = ld_bytes(V, (uint32_t)bb);
        acc += w[p] * (vf - vi);
        acc += w[np + p] * (vb - vi);
      };
      if constexpr (P > 0) {
#pragma unroll
        for (int p = 0; p < P; ++p) edge(p);
      } else {
        for (int p = 0; p < np; ++p) edge(p);
      }
      mv = w[2 * np];
    };
    if (__ballot(c != c0) == 0ull) {
      const T* w = a.ctab + (uint32_t)(c0 * a.tw);
      if (inner)
        sweep(w, NoClamp{});
      else
        sweep(w, Clamp{});
    } else {
      sweep(a.ctab + (uint32_t)(c * a.tw), Clamp{});
    }
    const T sr = active ? stimulus_sum(a, active, (int64_t)i) : T(0);
    *(T*)((char*)a.Vout + (uint32_t)bi) = vi + hT * (mv * acc + sr);
  }
}

// ---------------------------------------------------------------------------
// Stencil rows by class, neighbour rows shared across lanes (grid_rows.h).
// The arithmetic and its order are those of k_diff_classes, so the results
// are the same bits.  Each wavefront produces ITER consecutive groups of
// kWaveRows rows; the loads of all groups are issued before any group is
// computed.
// ---------------------------------------------------------------------------
// One potential by a raw buffer load at byte offset off (0 outside the
// buffer's range).
template <typename T>
__device__ __forceinline__ T ld_raw(__amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// One potential stored by a raw buffer store at byte offset off (dropped
// outside the buffer's range).
template <typename T>
__device__ __forceinline__ void st_raw(__amdgpu_buffer_rsrc_t r, uint32_t off, T v) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((__vector_size__(8))) unsigned int, v), r, (int)off, 0,
        0);
}

// Occupancy floor: in FP32 with one or two row groups per wavefront the
// kernel fits 64 registers without spilling, i.e. 8 wavefronts per SIMD (two
// groups otherwise take 66 registers and 7 wavefronts, 2% slower per launch
// on the 3D slab); four groups would spill under the floor, FP64 needs more.
template <typename T, int ITER>
constexpr int kRowsWavesPerEU = (sizeof(T) == 4 && ITER <= 2) ? 8 : 1;

template <typename T, int P, int BLOCK, int ITER>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(kRowsWavesPerEU<T, ITER>))) void k_diff_rows(
    DiffArgs<T> a, const T* __restrict__ ctab, const int32_t* __restrict__ wcls) {
  using RP = RowPattern<P>;
  constexpr int NC = RP::NC;
  constexpr int WR = kWaveRows;
  constexpr int WPB = BLOCK / 64;
  constexpr int ES = (int)sizeof(T);
  const int n = (int)a.n;
  const int64_t ngroups = (a.n + WR - 1) / WR;
  const int64_t nb = (ngroups + (int64_t)WPB * ITER - 1) / ((int64_t)WPB * ITER);
  const int lane = threadIdx.x & 63;
  // first row group of this wavefront (wave-uniform)
  const int64_t g0 =
      (row_block(nb, a.xcd) * WPB + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6)) *
      ITER;
  if (g0 >= ngroups) return;                // whole wavefront past the end
  // row centres (kernel arguments, so the loads below need no memory
  // round trip for their addresses; validated on the host)
  int ctr[NC];
  ctr[0] = 0;
  if constexpr (P == 4) {
    ctr[1] = a.nx;
    ctr[2] = -a.nx;
  } else if constexpr (P == 13) {
    const int nx = a.nx, nxy = a.nxy;
    ctr[1] = nx;
    ctr[2] = nxy - nx;
    ctr[3] = nxy;
    ctr[4] = nxy + nx;
    for (int k = 1; k < 5; ++k) ctr[4 + k] = -ctr[k];
  }
  // every lane (halo lanes included) loads the centre rows of every group;
  // all lanes stay active through the shifts.  Raw buffer loads over the n
  // potentials: an index outside [0, n) (before the first or past the last
  // row) reads 0 with no clamp arithmetic; such a value only ever meets a
  // zero weight (no element joins a row to a node across the grid's ends).
  const __amdgpu_buffer_rsrc_t vres =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.Vin, (short)0, n * ES, 0x00020000);
  int cb[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) cb[k] = ctr[k] * ES;
  T vc[ITER][NC];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int ib = ((int)((g0 + it) * WR) + lane - 1) * ES;
#pragma unroll
    for (int k = 0; k < NC; ++k) vc[it][k] = ld_raw<T>(vres, ib + cb[k]);
  }
  const double dt_ad = a.dt_ad[0];
  const T hT = (T)dt_ad;
  const uint32_t active = open_stimuli(a, dt_ad);
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int64_t g = g0 + it;
    if (g >= ngroups) break;
    const int i = (int)(g * WR) + lane - 1;
    const bool produce = lane >= 1 && lane <= WR && i < n;
    // the shifts are taken where each neighbour is used (once per path), so
    // the compiler can fold each into the subtraction that consumes it
    auto pick = [&](int k, int d) -> T {
      return d > 0 ? lane_shift<1>(vc[it][k]) : (d < 0 ? lane_shift<-1>(vc[it][k]) : vc[it][k]);
    };
    const T vi = vc[it][0];
    T acc = T(0), mv;
    auto sweep = [&](auto w) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const T vf = pick(RP::fk(p), RP::fd(p));
        const T vb = pick(RP::bk(p), RP::bd(p));
        acc += w[p] * (vf - vi);
        acc += w[P + p] * (vb - vi);
      }
      mv = w[2 * P];
    };
    // class shared by the group's rows, or kNoClass
    const int wc = wcls[g];
    if (wc != kNoClass) {
      // one table row for the whole wavefront: read through the constant
      // address space, i.e. by scalar loads
      using CT = const __attribute__((address_space(4))) T*;
      sweep((CT)(ctab + (uint32_t)(wc * a.tw)));
    } else {
      const int ic = min(max(i, 0), n - 1);
      sweep(ctab + (uint32_t)((int)a.cls[(uint32_t)ic] * a.tw));
    }
    if (produce) {
      const T sr = active ? stimulus_sum(a, active, (int64_t)i) : T(0);
      *(T*)((char*)a.Vout + (uint32_t)(i * ES)) = vi + hT * (mv * acc + sr);
    }
  }
}

// ---------------------------------------------------------------------------
// L consecutive substeps (a.m .. a.m + L - 1 of a half step) in one launch, for
// structured 3D grids with row classes and one instance: temporal blocking.
// A workgroup owns a tile of 64 - 2L consecutive x, ty = 16 - 2L y rows and
// tz z planes.  Its 16 wavefronts are the tile's y rows widened by L on each
// side (a wavefront's lanes cover x - L .. x + 63 - L), and together they
// march z through the tile's planes widened by L.  Level t (the potential
// after t of the L substeps) of a plane is computed as soon as level t - 1
// holds the plane after it: from level t - 1 of the three planes around it,
// of which each wavefront keeps its own row in registers and shares it with
// the rows above and below through a ring of three planes per level in LDS;
// x-neighbours come from adjacent lanes (DPP) as in the row-sharing kernel.
// Level t is exact on a region one node smaller on every side than level
// t - 1, so after L levels the tile's own nodes are.  Nodes outside the grid
// hold 0; the host admits a grid only when no weight joins a node to a
// position outside it (row ends, faces), so those zeros only ever meet zero
// weights, as the wrapped neighbours of the row-sharing kernel do.  Every
// node's arithmetic (weights, order, stimulus) is that of k_diff_rows: for
// finite potentials the result is the same bits as L launches of it.
// ---------------------------------------------------------------------------
constexpr int kFusedClassSweeps = 4;

template <typename T, int L>
__global__ __launch_bounds__(kFusedRows * 64) void k_diff_fused(DiffArgs<T> a,
                                                                const T* __restrict__ ctab,
                                                                FusedGeom g) {
  constexpr int P = 13;
  constexpr int NY = kFusedRows;           // wavefronts = y rows of the window
  constexpr int W = 64;
  constexpr int PF = 3;                    // planes loaded ahead of their use
  using RP = RowPattern<P>;
  __shared__ T ring[L][3][NY][W];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  int b = blockIdx.x;
  const int xs = b % g.nxs;
  b /= g.nxs;
  const int ys = b % g.nys;
  const int zs = b / g.nys;
  const int x = xs * (W - 2 * L) - L + lane;
  const int y = ys * (NY - 2 * L) - L + wv;  // wavefront-uniform
  const int NZ = g.tz + 2 * L;
  const int z0 = zs * g.tz - L;
  const bool xin = x >= 0 && x < g.nx;
  const bool yin = y >= 0 && y < g.ny;
  const int nxy = g.nx * g.ny;
  const double dt_ad = a.dt_ad[0];
  const T hT = (T)dt_ad;
  const bool stim = a.stim_mask != nullptr;
  uint32_t open[L];                        // stimuli open on each substep
#pragma unroll
  for (int t = 0; t < L; ++t) open[t] = open_stimuli_at(a, dt_ad, a.m + t);
  // Loads and the final store go through buffer resources over the n rows:
  // a node outside the grid takes an offset past the end, which reads 0 and
  // drops the store, so no access depends on a branch and the loads of later
  // planes stay in flight across the levels.
  const int n = (int)a.n;
  constexpr int ES = (int)sizeof(T);
  constexpr uint32_t kOut = 0x80000000u;   // past every buffer (n * ES < 2^31)
  const __amdgpu_buffer_rsrc_t rv =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.Vin, (short)0, n * ES, 0x00020000);
  const __amdgpu_buffer_rsrc_t ro =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.Vout, (short)0, n * ES, 0x00020000);
  const __amdgpu_buffer_rsrc_t rc =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.cls, (short)0, n * 2, 0x00020000);
  const __amdgpu_buffer_rsrc_t rm =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.stim_mask, (short)0, stim ? n : 0, 0x00020000);
  // this lane's node of window plane zz: value, class and stimulus mask
  auto fetch = [&](int zz, T& v, unsigned short& c, unsigned char& mk) {
    const int z = z0 + zz;
    const bool in = zz < NZ && xin && yin && z >= 0 && z < g.nz;
    const uint32_t i = in ? (uint32_t)(x + g.nx * y + nxy * z) : kOut;
    v = ld_raw<T>(rv, (int)(in ? i * (uint32_t)ES : kOut));
    c = __builtin_amdgcn_raw_buffer_load_b16(rc, (int)(in ? 2u * i : kOut), 0, 0);
    mk = __builtin_amdgcn_raw_buffer_load_b8(rm, (int)i, 0, 0);
  };
  // planes s, s+1, s+2 in flight, plane s in slot s % 3 (the march is
  // unrolled by 3, so no loaded register is ever moved: a move would wait for
  // its load)
  T pv[PF];
  unsigned short pc[PF];
  unsigned char pm[PF];
#pragma unroll
  for (int q = 0; q < PF; ++q) fetch(q, pv[q], pc[q], pm[q]);
  // own row: level t of plane p in own[t][p % 3]
  T own[L][3];
  int cr[L + 1];          // class and stimulus mask of this lane's node at
  uint32_t mr[L + 1];     // planes s, s-1, ..., s-L
#pragma unroll
  for (int t = 0; t < L; ++t) own[t][0] = own[t][1] = own[t][2] = T(0);
#pragma unroll
  for (int j = 0; j <= L; ++j) {
    cr[j] = 0;
    mr[j] = 0u;
  }
  auto plane = [&](int s, auto U) {
    constexpr int u = decltype(U)::value;   // s % 3
    // level 0 of plane s, and the load of plane s + 3 into its slot
#pragma unroll
    for (int j = L; j > 0; --j) {
      cr[j] = cr[j - 1];
      mr[j] = mr[j - 1];
    }
    cr[0] = (int)pc[u];
    mr[0] = (uint32_t)pm[u];
    own[0][u] = pv[u];
    ring[0][u][wv][lane] = pv[u];
    fetch(s + PF, pv[u], pc[u], pm[u]);     // past the window: no access, 0
    __syncthreads();
#pragma unroll
    for (int t = 1; t <= L; ++t) {
      const int zz = s - t;
      // ring slots of planes zz - 1, zz, zz + 1
      const int s0 = (u - t % 3 + 3) % 3, sm = (s0 + 2) % 3, sp = (s0 + 1) % 3;
      T out = T(0);
      T vL = T(0);                           // level L: the value and where it goes
      uint32_t offL = kOut;
      if (zz >= t && zz < NZ - t && wv >= t && wv < NY - t) {
        const int z = z0 + zz;
        const bool in = xin && yin && z >= 0 && z < g.nz;
        // level t-1 around (zz, this row): the row centres of RowPattern<13>
        // (0; y+1; z+1 y-1; z+1; z+1 y+1; y-1; z-1 y+1; z-1; z-1 y-1)
        T vc[9];
        vc[0] = own[t - 1][s0];
        vc[1] = ring[t - 1][s0][wv + 1][lane];
        vc[2] = ring[t - 1][sp][wv - 1][lane];
        vc[3] = own[t - 1][sp];
        vc[4] = ring[t - 1][sp][wv + 1][lane];
        vc[5] = ring[t - 1][s0][wv - 1][lane];
        vc[6] = ring[t - 1][sm][wv + 1][lane];
        vc[7] = own[t - 1][sm];
        vc[8] = ring[t - 1][sm][wv - 1][lane];
        auto pick = [&](int k, int d) -> T {
          return d > 0 ? lane_shift<1>(vc[k]) : (d < 0 ? lane_shift<-1>(vc[k]) : vc[k]);
        };
        const T vi = vc[0];
        T df[P], db[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          df[p] = pick(RP::fk(p), RP::fd(p)) - vi;
          db[p] = pick(RP::bk(p), RP::bd(p)) - vi;
        }
        auto sweep = [&](auto w) {
          T acc = T(0);
#pragma unroll
          for (int p = 0; p < P; ++p) {
            acc += w[p] * df[p];
            acc += w[P + p] * db[p];
          }
          return acc;
        };
        // weights by class: one sweep per class among the nodes this level
        // keeps, its table row read by scalar loads, each lane taking the
        // sweep of its own class; lanes left after kFusedClassSweeps classes
        // read their rows per lane
        const int c = cr[t];
        const bool keep = in && lane >= t && lane < W - t;
        unsigned long long rem = __ballot(keep);
        T acc = T(0), mv = T(0);
        for (int q = 0; q < kFusedClassSweeps && rem; ++q) {
          const int cu = __builtin_amdgcn_readlane(c, __ffsll((long long)rem) - 1);
          using CT = const __attribute__((address_space(4))) T*;
          const CT w = (CT)(ctab + (uint32_t)(cu * a.tw));
          const T r = sweep(w);
          const T m = w[2 * P];
          // lanes of this class, taken from the ballot (so that the sweep
          // keeps its scalar table row)
          const unsigned long long mm = __ballot(c == cu);
          const bool mine = (mm >> lane) & 1ull;
          acc = mine ? r : acc;
          mv = mine ? m : mv;
          rem &= ~mm;
        }
        if (rem) {
          const T* w = ctab + (uint32_t)(c * a.tw);
          const T r = sweep(w);
          const T m = w[2 * P];
          const bool left = (rem >> lane) & 1ull;
          acc = left ? r : acc;
          mv = left ? m : mv;
        }
        T sr = T(0);
        const uint32_t mk = mr[t] & open[t - 1];
        if (mk)
          for (int q = 0; q < a.stim.n; ++q)
            if (mk & (1u << q)) sr += (T)a.stim.amp[q];
        const T v = vi + hT * (mv * acc + sr);
        out = in ? v : T(0);
        if (t < L) {
          ring[t][s0][wv][lane] = out;
        } else {
          // the tile's own nodes (wv and zz are wavefront-uniform)
          const bool own_node = in && lane >= L && lane < W - L && wv >= L && wv < NY - L &&
                                zz >= L && zz < NZ - L;
          vL = v;
          offL = own_node ? (uint32_t)(x + g.nx * y + nxy * z) * (uint32_t)ES : kOut;
        }
      }
      if (t < L) {
        own[t][s0] = out;
        __syncthreads();
      } else {
        // one store per plane and lane, outside the branch (dropped off the
        // tile), so that every plane issues the same memory operations
        st_raw<T>(ro, offL, vL);
      }
    }
  };
  for (int s = 0; s < NZ; s += 3) {
    plane(s, std::integral_constant<int, 0>{});
    if (s + 1 < NZ) plane(s + 1, std::integral_constant<int, 1>{});
    if (s + 2 < NZ) plane(s + 2, std::integral_constant<int, 2>{});
  }
}

template <typename T, int L>
static void launch_fused_k(const DiffArgs<T>& a, const FusedGeom& g, hipStream_t s) {
  const dim3 grid((unsigned)(g.nxs * g.nys * g.nzs));
  launch_step_kernel(k_diff_fused<T, L>, grid, dim3(kFusedRows * 64), s, a, a.ctab, g);
}

template <typename T>
void launch_diffusion_fused(const DiffArgs<T>& a, int L, const FusedGeom& g, hipStream_t s) {
  if (a.n <= 0) return;
  switch (L) {
    case 2: launch_fused_k<T, 2>(a, g, s); return;
    case 3: launch_fused_k<T, 3>(a, g, s); return;
    default: launch_fused_k<T, 4>(a, g, s); return;
  }
}
template void launch_diffusion_fused<float>(const DiffArgs<float>&, int, const FusedGeom&,
                                            hipStream_t);
template void launch_diffusion_fused<double>(const DiffArgs<double>&, int, const FusedGeom&,
                                             hipStream_t);

template <typename T, int P, int BLOCK, int ITER>
static void launch_rows_k(const DiffArgs<T>& a, hipStream_t s) {
  const int64_t ngroups = (a.n + kWaveRows - 1) / kWaveRows;
  const int64_t per = (int64_t)(BLOCK / 64) * ITER;
  const dim3 grid((unsigned)((ngroups + per - 1) / per));
  launch_step_kernel(k_diff_rows<T, P, BLOCK, ITER>, grid, dim3(BLOCK), s, a, a.ctab, a.wcls);
}
template <typename T, int P, int BLOCK>
static void launch_rows_i(const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (c.diff_rpl == 2) return launch_rows_k<T, P, BLOCK, 2>(a, s);
  if (c.diff_rpl >= 4) return launch_rows_k<T, P, BLOCK, 4>(a, s);
  launch_rows_k<T, P, BLOCK, 1>(a, s);
}
template <typename T, int P>
static void launch_rows_b(const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (c.diff_block == 128) return launch_rows_i<T, P, 128>(a, c, s);
  if (c.diff_block == 512) return launch_rows_i<T, P, 512>(a, c, s);
  launch_rows_i<T, P, 256>(a, c, s);
}

template <typename T, int P, int BLOCK, int ITER>
static void launch_classes_k(const DiffArgs<T>& a, hipStream_t s) {
  const int64_t per = (int64_t)BLOCK * ITER;
  const dim3 grid((unsigned)((a.n + per - 1) / per));
  launch_step_kernel(k_diff_classes<T, P, BLOCK, ITER>, grid, dim3(BLOCK), s, a);
}
template <typename T, int P, int BLOCK>
static void launch_classes_i(const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  switch (c.diff_rpl) {
    case 2: return launch_classes_k<T, P, BLOCK, 2>(a, s);
    case 4: return launch_classes_k<T, P, BLOCK, 4>(a, s);
    case 8: return launch_classes_k<T, P, BLOCK, 8>(a, s);
    case 16: return launch_classes_k<T, P, BLOCK, 16>(a, s);
    default: return launch_classes_k<T, P, BLOCK, 1>(a, s);
  }
}
template <typename T, int P>
static void launch_classes_b(const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (c.diff_block == 128) return launch_classes_i<T, P, 128>(a, c, s);
  if (c.diff_block == 512) return launch_classes_i<T, P, 512>(a, c, s);
  launch_classes_i<T, P, 256>(a, c, s);
}

template <typename T, int P, bool BATCHED, int BLOCK, int RPL>
static void launch_stencil_k(const DiffArgs<T>& a, hipStream_t s) {
  const int64_t nlanes = (a.n + RPL - 1) / RPL;
  const dim3 grid((unsigned)((nlanes + BLOCK - 1) / BLOCK));
  if (a.Np * (int64_t)sizeof(T) < (int64_t(1) << 31))
    launch_step_kernel(k_diff_stencil<T, P, BATCHED, BLOCK, RPL, true>, grid, dim3(BLOCK), s, a);
  else
    launch_step_kernel(k_diff_stencil<T, P, BATCHED, BLOCK, RPL, false>, grid, dim3(BLOCK), s, a);
}

template <typename T, int P, bool BATCHED, int BLOCK>
static void launch_stencil_r(const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (c.diff_rpl == 4) return launch_stencil_k<T, P, BATCHED, BLOCK, 4>(a, s);
  }
  if (c.diff_rpl == 2) return launch_stencil_k<T, P, BATCHED, BLOCK, 2>(a, s);
  launch_stencil_k<T, P, BATCHED, BLOCK, 1>(a, s);
}

template <typename T, int P, bool BATCHED>
static void launch_stencil_b(const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (c.diff_block == 128) return launch_stencil_r<T, P, BATCHED, 128>(a, c, s);
  if (c.diff_block == 512) return launch_stencil_r<T, P, BATCHED, 512>(a, c, s);
  launch_stencil_r<T, P, BATCHED, 256>(a, c, s);
}

template <typename T, int P>
static void launch_stencil_p(const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (a.inst)
    launch_stencil_b<T, P, true>(a, c, s);
  else
    launch_stencil_b<T, P, false>(a, c, s);
}

template <typename T, bool BATCHED, int BLOCK>
static void launch_ell_k(const DiffArgs<T>& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + BLOCK - 1) / BLOCK));
  // widths of the element types on structured and split grids
  switch (a.W) {
    case 2: return launch_step_kernel(k_diff_ell<T, BATCHED, BLOCK, 2>, grid, dim3(BLOCK), s, a);
    case 6: return launch_step_kernel(k_diff_ell<T, BATCHED, BLOCK, 6>, grid, dim3(BLOCK), s, a);
    case 8: return launch_step_kernel(k_diff_ell<T, BATCHED, BLOCK, 8>, grid, dim3(BLOCK), s, a);
    case 14: return launch_step_kernel(k_diff_ell<T, BATCHED, BLOCK, 14>, grid, dim3(BLOCK), s, a);
    case 26: return launch_step_kernel(k_diff_ell<T, BATCHED, BLOCK, 26>, grid, dim3(BLOCK), s, a);
    default: return launch_step_kernel(k_diff_ell<T, BATCHED, BLOCK, 0>, grid, dim3(BLOCK), s, a);
  }
}
template <typename T, bool BATCHED>
static void launch_ell_b(const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (c.diff_block == 128) return launch_ell_k<T, BATCHED, 128>(a, s);
  if (c.diff_block == 512) return launch_ell_k<T, BATCHED, 512>(a, s);
  launch_ell_k<T, BATCHED, 256>(a, s);
}

template <typename T>
void launch_diffusion(int layout, const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (a.n <= 0) return;
  if (layout == MONO_LAYOUT_ELL) {
    if (a.inst)
      launch_ell_b<T, true>(a, c, s);
    else
      launch_ell_b<T, false>(a, c, s);
    return;
  }
  if (a.cls && !a.inst && c.diff_classes && a.n * (int64_t)sizeof(T) < (int64_t(1) << 31)) {
    if (a.wcls && c.diff_wave_rows) {
      switch (a.P) {
        case 1: launch_rows_b<T, 1>(a, c, s); return;
        case 4: launch_rows_b<T, 4>(a, c, s); return;
        case 13: launch_rows_b<T, 13>(a, c, s); return;
        default: break;
      }
    }
    switch (a.P) {
      case 1: launch_classes_b<T, 1>(a, c, s); break;
      case 4: launch_classes_b<T, 4>(a, c, s); break;
      case 13: launch_classes_b<T, 13>(a, c, s); break;
      default: launch_classes_b<T, 0>(a, c, s); break;
    }
    return;
  }
  switch (a.P) {
    case 1: launch_stencil_p<T, 1>(a, c, s); break;
    case 4: launch_stencil_p<T, 4>(a, c, s); break;
    case 13: launch_stencil_p<T, 13>(a, c, s); break;
    default: launch_stencil_p<T, 0>(a, c, s); break;
  }
}

template void launch_diffusion<float>(int, const DiffArgs<float>&, const LaunchCfg&, hipStream_t);
template void launch_diffusion<double>(int, const DiffArgs<double>&, const LaunchCfg&,
                                       hipStream_t);

__global__ void k_advance_clock(int64_t* base, int64_t by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *base += by;
}
void launch_advance_clock(int64_t* base, int64_t by, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_clock, dim3(1), dim3(64), 0, s, base, by);
}
__global__ void k_set_clock(int64_t* base, int64_t to) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *base = to;
}
void launch_set_clock(int64_t* base, int64_t to, hipStream_t s) {
  hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, s, base, to);
}

// ---------------------------------------------------------------------------
// eq. (3): Gershgorin rows in FP64
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gersh_rows(int64_t n, const int64_t* rp,
                                                       const int32_t* col, const double* val,
                                                       const double* mass, double* r,
                                                       double* g) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double kii = 0.0, off = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
    const double v = val[p];
    if (col[p] == i)
      kii += v;
    else
      off += fabs(v);
  }
  const double s = kii + off;
  r[i] = mass[i] / s;
  g[i] = s / mass[i];
}

void launch_gershgorin(int64_t n, const int64_t* rp, const int32_t* col, const double* val,
                       const double* mass, double* r, double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_gersh_rows, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, n, rp, col, val, mass, r, g);
}

// wavefront (64-lane) reductions through cross-lane shuffles
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One workgroup per instance: min of r and max of g over its rows.
__global__ __launch_bounds__(kBlock) void k_seg_minmax(const int64_t* inst_off, const double* r,
                                                       const double* g, double* rmin,
                                                       double* gmax) {
  __shared__ double smin[kBlock / 64], smax[kBlock / 64];
  const int q = blockIdx.x;
  double mn = INFINITY, mx = 0.0;
  for (int64_t i = inst_off[q] + threadIdx.x; i < inst_off[q + 1]; i += kBlock) {
    mn = fmin(mn, r[i]);
    mx = fmax(mx, g[i]);
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    smin[w] = mn;
    smax[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBlock / 64; ++k) {
      mn = fmin(mn, smin[k]);
      mx = fmax(mx, smax[k]);
    }
    rmin[q] = mn;
    gmax[q] = mx;
  }
}

void launch_segmented_minmax(int n_inst, const int64_t* inst_off, const double* r,
                             const double* g, double* rmin, double* gmax, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_minmax, dim3(n_inst), dim3(kBlock), 0, s, inst_off, r, g, rmin, gmax);
}

// ---------------------------------------------------------------------------
// power iteration for lambda_max(M_L^-1 K), FP64 (diagnostic)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_spmv_csr(int64_t n, const int64_t* rp,
                                                     const int32_t* col, const double* val,
                                                     const double* x, double* y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += val[p] * x[col[p]];
  y[i] = s;
}
void launch_spmv_csr(int64_t n, const int64_t* rp, const int32_t* col, const double* val,
                     const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv_csr, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     n, rp, col, val, x, y);
}

__global__ __launch_bounds__(kBlock) void k_seg_dots(const int64_t* inst_off, const double* x,
                                                     const double* kx, const double* mass,
                                                     double* xkx, double* xmx) {
  __shared__ double sa[kBlock / 64], sb[kBlock / 64];
  const int q = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = inst_off[q] + threadIdx.x; i < inst_off[q + 1]; i += kBlock) {
    a += x[i] * kx[i];
    b += x[i] * mass[i] * x[i];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBlock / 64; ++k) {
      a += sa[k];
      b += sb[k];
    }
    xkx[q] = a;
    xmx[q] = b;
  }
}
void launch_segmented_dots(int n_inst, const int64_t* inst_off, const double* x, const double* kx,
                           const double* mass, double* xkx, double* xmx, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_dots, dim3(n_inst), dim3(kBlock), 0, s, inst_off, x, kx, mass, xkx,
                     xmx);
}

// x <- (M^-1 K x) / ||x||_M of its instance (xmx = x^T M x per instance)
__global__ __launch_bounds__(kBlock) void k_power_update(int64_t n, const int32_t* inst,
                                                         const double* kx, const double* mass,
                                                         const double* xmx, double* x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int q = inst ? inst[i] : 0;
  x[i] = kx[i] / mass[i] / sqrt(xmx[q]);
}
void launch_power_update(int64_t n, const int32_t* inst, const double* kx, const double* mass,
                         const double* xmx, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_power_update, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, n, inst, kx, mass, xmx, x);
}

// deterministic start vector with energy in every mode (integer hash in [-1,1])
__global__ __launch_bounds__(kBlock) void k_power_init(int64_t n, double* x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
void launch_power_init(int64_t n, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_power_init, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, n, x);
}

// precision conversion helpers
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_f64(int64_t n, const T* src, double* dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_from_f64(int64_t n, const double* src, T* dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}
template <typename T>
void launch_convert(int64_t n, const T* src, double* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_to_f64<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, n, src, dst);
}
template <typename T>
void launch_convert_from(int64_t n, const double* src, T* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_from_f64<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, n, src, dst);
}
template void launch_convert<float>(int64_t, const float*, double*, hipStream_t);
template void launch_convert<double>(int64_t, const double*, double*, hipStream_t);
template void launch_convert_from<float>(int64_t, const double*, float*, hipStream_t);
template void launch_convert_from<double>(int64_t, const double*, double*, hipStream_t);

}  // namespace mono
