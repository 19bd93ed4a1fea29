// cg_kernels.hip - gfx950 kernels of the stencil conjugate-gradient library.
//
// The method (arXiv 1803.03797): conjugate gradients on the Laplacian of
// Section II, with the matrix-vector product applied as the 5-point stencil of
// Section II-B (never assembled), in the two variants of the paper:
// Algorithm 1 (stdCG) and Algorithm 2 (newCG, the pipelined CG that lets the
// stencil and the two dot products proceed together, Section II dataflow
// discussion).  The FPGA design of the paper (line buffers, FACTOR-way
// superscalar streams, padding copies) is replaced by a GPU design:
//
//  * Every CG step is a "pass" over the grid that fuses the stencil with the
//    dot products and axpy updates of that step (Section II-C: dot product and
//    axpy blocks), so each vector crosses HBM once per pass.
//  * A pass walks tiles; inside a tile each wavefront marches down a strip of
//    rows keeping the south/centre/north rows of the halo vector in registers;
//    west/east neighbours come from adjacent lanes through wavefront-wide DPP
//    shifts, and the tile's outer columns from one extra load per edge lane.
//  * Dot products use a fixed order: per-lane fma accumulation in row order,
//    xor butterfly across the 64 lanes, wavefronts in order, one FP64 partial
//    per tile; the next pass sums the partials in tile order (every
//    work-group redundantly, so no atomics or cross-work-group fences are
//    needed) and evaluates the scalar recurrences of the algorithm before its
//    own body.  Results are bitwise reproducible.
//
// All arithmetic is written with explicit fma() where the contract says fma;
// the library is built with -ffp-contract=off so nothing else is fused.
#include <math.h>

#include <type_traits>
#include <utility>

#include "cg_internal.h"

namespace cgk {

// ------------------------------------------------------------- lane rows --

template <typename T, int CPL>
struct Row {
  T e[CPL];
};

template <typename T, int CPL>
__device__ __forceinline__ Row<T, CPL> zrow() {
  Row<T, CPL> v;
#pragma unroll
  for (int k = 0; k < CPL; ++k) v.e[k] = T(0);
  return v;
}

template <typename T, int CPL>
__device__ __forceinline__ Row<T, CPL> ldrow(const T* p) {
  Row<T, CPL> v;
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int k = 0; k < CPL; k += 2) {
      double2 t = *reinterpret_cast<const double2*>(p + k);
      v.e[k] = t.x;
      v.e[k + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < CPL; k += 4) {
      float4 t = *reinterpret_cast<const float4*>(p + k);
      v.e[k] = t.x;
      v.e[k + 1] = t.y;
      v.e[k + 2] = t.z;
      v.e[k + 3] = t.w;
    }
  }
  return v;
}

// Stores the first `valid` elements (valid >= CPL: the whole row segment).
template <typename T, int CPL>
__device__ __forceinline__ void strow(T* p, const Row<T, CPL>& v, int valid) {
  if (valid >= CPL) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int k = 0; k < CPL; k += 2)
        *reinterpret_cast<double2*>(p + k) = make_double2(v.e[k], v.e[k + 1]);
    } else {
#pragma unroll
      for (int k = 0; k < CPL; k += 4)
        *reinterpret_cast<float4*>(p + k) =
            make_float4(v.e[k], v.e[k + 1], v.e[k + 2], v.e[k + 3]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < CPL; ++k)
      if (k < valid) p[k] = v.e[k];
  }
}

// ---------------------------------------------------- wavefront exchange --

constexpr int kDppWaveShr1 = 0x138;  // lane l receives lane l-1 (lane 0 keeps `old`)
constexpr int kDppWaveShl1 = 0x130;  // lane l receives lane l+1 (lane 63 keeps `old`)

template <int CTRL>
__device__ __forceinline__ double dpp(double v, double old) {
  int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, 0xf, 0xf,
                                       false);
  int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, 0xf, 0xf,
                                       false);
  return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v, float old) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                    0xf, 0xf, false));
}

// West and east neighbours of every element of a lane's row segment.  eW is
// the value left of the tile (used by lane 0), eE the value right of it
// (used by lane 63).  Must be called with the whole wavefront active.
template <typename T, int CPL>
__device__ __forceinline__ void west_east(const Row<T, CPL>& v, T eW, T eE, Row<T, CPL>& W,
                                          Row<T, CPL>& E) {
  W.e[0] = dpp<kDppWaveShr1>(v.e[CPL - 1], eW);
  E.e[CPL - 1] = dpp<kDppWaveShl1>(v.e[0], eE);
#pragma unroll
  for (int k = 1; k < CPL; ++k) W.e[k] = v.e[k - 1];
#pragma unroll
  for (int k = 0; k < CPL - 1; ++k) E.e[k] = v.e[k + 1];
}

// (A u) at one point: (((4 uC - uW) - uE) - uS) - uN, S = row j-1, N = row j+1.
template <typename T>
__device__ __forceinline__ T st5(T c, T w, T e, T s, T n) {
  return (((T(4) * c - w) - e) - s) - n;
}

// The operator at one point, selected by OP:
//   0: the 5-point stencil;
//   1: the 7-point one in 3D, (((((6 uC - uW) - uE) - uS) - uN) - uB) - uT,
//      B = plane l-1, T = plane l+1;
//   2: the variable-coefficient 5-point one with face conductivities kw, ke,
//      ks, kn: d = ((kw + ke) + ks) + kn, then (((d uC - kw uW) - ke uE) -
//      ks uS) - kn uN, each product rounded before its subtraction.
template <int OP, typename T>
__device__ __forceinline__ T stn(T c, T w, T e, T s, T n, T b, T t, T kw, T ke, T ks, T kn) {
  if constexpr (OP == 1) {
    return (((((T(6) * c - w) - e) - s) - n) - b) - t;
  } else if constexpr (OP == 2) {
    const T d = ((kw + ke) + ks) + kn;
    const T pc = d * c, pw = kw * w, pe = ke * e, ps = ks * s, pn = kn * n;
    return (((pc - pw) - pe) - ps) - pn;
  } else {
    return st5(c, w, e, s, n);
  }
}

// The four face conductivities of a lane's cells on one row.
template <typename T, int CPL>
struct Kc {
  Row<T, CPL> w, e, s, n;
};

// The operator at column k of a lane's row from the walker's rows.
template <int OP, typename T, int CPL, class KC>
__device__ __forceinline__ T op_at(const Row<T, CPL>& S, const Row<T, CPL>& C,
                                   const Row<T, CPL>& N, const Row<T, CPL>& W,
                                   const Row<T, CPL>& E, const Row<T, CPL>& B,
                                   const Row<T, CPL>& U, const KC& kc, int k) {
  if constexpr (OP == 2) {
    return stn<2>(C.e[k], W.e[k], E.e[k], S.e[k], N.e[k], T(0), T(0), kc.w.e[k], kc.e.e[k],
                  kc.s.e[k], kc.n.e[k]);
  } else {
    return stn<OP>(C.e[k], W.e[k], E.e[k], S.e[k], N.e[k], B.e[k], U.e[k], T(0), T(0), T(0),
                   T(0));
  }
}

// Reads a State every lane needs with the same value into scalar registers
// (readfirstlane), so the solve's scalars do not hold vector registers (which
// the compiler would otherwise spill across the prologue's barriers).
__device__ __forceinline__ State load_state_uniform(const State* p) {
  static_assert(sizeof(State) % 16 == 0, "State is loaded as uint4");
  constexpr int N = sizeof(State) / 4;
  uint32_t u[N];
  const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
  for (int i = 0; i < N / 4; ++i) {
    const uint4 v = q[i];
    u[4 * i + 0] = __builtin_amdgcn_readfirstlane(v.x);
    u[4 * i + 1] = __builtin_amdgcn_readfirstlane(v.y);
    u[4 * i + 2] = __builtin_amdgcn_readfirstlane(v.z);
    u[4 * i + 3] = __builtin_amdgcn_readfirstlane(v.w);
  }
  State s;
  __builtin_memcpy(&s, u, sizeof(State));
  return s;
}

// The same for a State held in registers whose fields are uniform (all
// threads computed them from the same sums).
__device__ __forceinline__ State uniform_state(const State& in) {
  constexpr int N = sizeof(State) / 4;
  uint32_t u[N];
  __builtin_memcpy(u, &in, sizeof(State));
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = __builtin_amdgcn_readfirstlane(u[i]);
  State s;
  __builtin_memcpy(&s, u, sizeof(State));
  return s;
}

__device__ __forceinline__ double uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = v + __shfl_xor(v, m, kWave);
  return v;
}

// The same butterfly (stage order 32, 16, ..., 1; every lane adds its xor
// partner) with the stages inside 32-lane halves done by DPP row/quad
// permutations (xor 8, 2, 1) or ds_swizzle (xor 16, 4), whose lane patterns
// are immediates: no per-lane address registers, half the LDS round trips.
template <int M>
__device__ __forceinline__ double swz_xor(double v) {
  constexpr int pat = 0x1f | (M << 10);  // bitmask mode: lane ^ M within 32 lanes
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), pat);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), pat);
  return __hiloint2double(hi, lo);
}

// DPP controls that are xor permutations inside 16-lane rows.
constexpr int kDppXor8 = 0x128;  // row_ror:8: lane l of a 16-lane row gets lane l ^ 8
constexpr int kDppXor2 = 0x4E;   // quad_perm [2,3,0,1]: lane l gets lane l ^ 2
constexpr int kDppXor1 = 0xB1;   // quad_perm [1,0,3,2]: lane l gets lane l ^ 1

__device__ __forceinline__ double wave_sum_swz(double v) {
  v = v + __shfl_xor(v, 32, kWave);
  v = v + swz_xor<16>(v);
  v = v + dpp<kDppXor8>(v, v);
  v = v + swz_xor<4>(v);
  v = v + dpp<kDppXor2>(v, v);
  v = v + dpp<kDppXor1>(v, v);
  return v;
}

// ------------------------------------------------------- tile geometry --

struct Strip {
  int tx, lane, wave;
  int c;       // first column of this lane
  int ct;      // first column of the tile
  int j0, j1;  // rows of this wavefront's strip, j0, j0 + js, ... < j1; empty
               // when j0 >= j1
  int js;      // row step: 1, or the rows of a plane (3D z-march)
  int y;       // 3D: the wavefront's in-plane row (may lie past the plane)
  int z0, z1;  // 3D: the tile's planes [z0, z1), the same for its wavefronts
};

// 2D: tile t = ty * ntx + tx of 4 wavefronts x rows rows; wavefront w walks
// rows ty * th + w * rows + [0, rows).  3D (g.plane > 0, the z-march): tile
// t = (tz * nty + ty) * ntx + tx of 4 consecutive in-plane rows (one per
// wavefront: y = ty * 4 + w) by rows planes; wavefront w walks its row y
// through planes tz * rows + [0, rows), one plane (g.plane stored rows) per
// step.
template <int CPL>
__device__ __forceinline__ Strip strip_of(const Geo& g, int t) {
  Strip s;
  s.tx = t % g.ntx;
  const int ty = t / g.ntx;
  s.lane = threadIdx.x & (kWave - 1);
  s.wave = (threadIdx.x >> 6) & (kWavesPerTile - 1);
  s.ct = s.tx * (kWave * CPL);
  s.c = s.ct + s.lane * CPL;
  if (g.plane > 0) {
    const int pl = g.plane, nz = g.ny / pl;
    const int y = (ty % g.nty) * kWavesPerTile + s.wave;
    const int z0 = (ty / g.nty) * g.rows, z1 = min(z0 + g.rows, nz);
    s.js = pl;
    s.y = y;
    s.z0 = z0;
    s.z1 = z1;
    s.j0 = s.j1 = 0;
    if (y < pl) {
      s.j0 = z0 * pl + y;
      s.j1 = z1 * pl + y;
    }
    return s;
  }
  s.js = 1;
  s.y = s.z0 = s.z1 = 0;
  s.j0 = ty * g.th + s.wave * g.rows;
  s.j1 = min(s.j0 + g.rows, g.ny);
  return s;
}

// Values just outside the tile on one row (zero outside the grid: the pad
// columns are zero, and there is no tile beyond the last one).
template <typename T, int CPL>
__device__ __forceinline__ void edges(const T* row, const Strip& s, const Geo& g, T& eW, T& eE) {
  eW = T(0);
  eE = T(0);
  if (s.lane == 0 && s.tx > 0) eW = row[s.ct - 1];
  if (s.lane == kWave - 1 && s.tx + 1 < g.ntx) eE = row[s.ct + kWave * CPL];
}

// ---------------------------------------------------------- scalar step --


__device__ __forceinline__ int stop_code(double gamma, double thr, int k, int maxit, double tol) {
  if (!isfinite(gamma)) return ST_BREAKDOWN;
  if (gamma <= thr) return ST_OK;
  if (k >= maxit) return tol == 0.0 ? ST_OK : ST_NOT_CONVERGED;
  return ST_RUNNING;
}

// Applies the scalar recurrences that sit between the previous pass and this
// one.  `sum` holds the cross-tile sums of the previous pass's partials.
// Returns true when this pass's body must run.
template <int KIND>
__device__ __forceinline__ bool transition(State& s, const double* sum, Sc& sc) {
  sc.al = 0.0;
  sc.be = 0.0;
  sc.first = 0;
  sc.xu = 0;
  sc.inv = 0.0;
  sc.alp = 0.0;
  if constexpr (KIND == K_PCGX) {
    return transition<K_PCG>(s, sum, sc);
  } else if constexpr (KIND == K_CG2X) {
    return transition<K_CG2>(s, sum, sc);
  } else if constexpr (KIND == K_CG2FX) {
    return transition<K_CG2F>(s, sum, sc);
  } else if constexpr (KIND == K_APPLY || KIND == K_DOT || KIND == K_RESID) {
    return true;
  } else if constexpr (KIND == K_RRQ || KIND == K_RRZ) {
    return s.status == ST_RUNNING;
  } else if constexpr (KIND == K_INIT_R) {
    return s.status == ST_RUNNING;
  } else if constexpr (KIND == K_INIT_W) {
    if (s.status != ST_RUNNING) return false;
    s.bb = sum[1];
    s.thr = (s.tol * s.tol) * s.bb;
    s.flags &= ~F_BB_PENDING;
    if (s.bb == 0.0) s.status = ST_ZERO_RHS;
    return s.status == ST_RUNNING;
  } else if constexpr (KIND == K_INIT_WU) {
    return s.status == ST_RUNNING;
  } else if constexpr (KIND == K_CHEBW) {
    // Preconditioned pipelined CG: gamma = (r,u), delta = (w,u) and the stop
    // test on (r,r); first pass alpha = gamma/delta, later beta =
    // gamma/gamma_old, alpha = 1/(delta/gamma - beta/alpha_old).  gamma is
    // kept in gamma0 (State::gamma holds (r,r), the residual reported).
    if (s.status != ST_RUNNING) return false;
    const double gu = sum[0], du = sum[1], rr = sum[2];
    int st = stop_code(rr, s.thr, s.k, s.maxit, s.tol);
    double al = 0.0, be = 0.0;
    if (st == ST_RUNNING) {
      if (s.k == 0) {
        if (!(du > 0.0) || !isfinite(du)) st = ST_BREAKDOWN;
        else al = gu / du;
      } else {
        be = gu / s.gamma0;
        const double den = du / gu - be / s.alpha;
        if (!(den > 0.0) || !isfinite(den)) st = ST_BREAKDOWN;
        else al = 1.0 / den;
      }
    }
    s.gamma = rr;
    s.gamma0 = gu;
    s.delta = du;
    s.status = st;
    if (st != ST_RUNNING) return false;
    s.alpha = al;
    s.beta = be;
    s.k += 1;
    return true;
  } else if constexpr (KIND == K_PPCG) {
    // the scalars of this iteration were set by the Chebyshev pass before it
    if (s.status != ST_RUNNING) return false;
    sc.al = s.alpha;
    sc.be = s.beta;
    sc.first = s.k == 1;
    return true;
  } else if constexpr (KIND == K_PCG) {
    // Algorithm 2: gamma = (r,r), delta = (w,r); first pass alpha = gamma/delta,
    // later beta = gamma/gamma_old, alpha = 1/(delta/gamma - beta/alpha_old).
    if (s.status != ST_RUNNING) return false;
    const double gamma = sum[0], delta = sum[1];
    int st = stop_code(gamma, s.thr, s.k, s.maxit, s.tol);
    double al = 0.0, be = 0.0;
    if (st == ST_RUNNING) {
      if (s.k == 0) {
        if (!(delta > 0.0) || !isfinite(delta)) st = ST_BREAKDOWN;
        else al = gamma / delta;
        sc.first = 1;
      } else {
        be = gamma / s.gamma;
        const double den = delta / gamma - be / s.alpha;
        if (!(den > 0.0) || !isfinite(den)) st = ST_BREAKDOWN;
        else al = 1.0 / den;
      }
    }
    s.gamma = gamma;
    s.delta = delta;
    s.status = st;
    if (st != ST_RUNNING) return false;
    s.alpha = al;
    s.beta = be;
    s.k += 1;
    sc.al = al;
    sc.be = be;
    return true;
  } else if constexpr (KIND == K_CHEB) {
    // Preconditioned CG: the stop test on gamma = (r,r) of the current
    // residual (from the initial residual pass or classic pass 2, which also
    // brings (b,b) the first time), before z = M^-1 r is formed.
    if (s.status != ST_RUNNING) return false;
    const double gamma = sum[0];
    if (s.flags & F_BB_PENDING) {
      s.bb = sum[1];
      s.thr = (s.tol * s.tol) * s.bb;
      s.flags &= ~F_BB_PENDING;
      if (s.bb == 0.0) {
        s.status = ST_ZERO_RHS;
        return false;
      }
    }
    const int st = stop_code(gamma, s.thr, s.k, s.maxit, s.tol);
    s.gamma = gamma;
    s.status = st;
    return st == ST_RUNNING;
  } else if constexpr (KIND == K_CG1) {
    // Algorithm 1: beta = (r,r)_new / (r,r)_old, then p = r + beta p.
    // Preconditioned: the one slot is rho = (r,z) from the Chebyshev pass
    // (which already made the stop test); beta = rho_new / rho_old with rho
    // kept in delta, then p = z + beta p.
    if (s.status != ST_RUNNING) return false;
    const double gamma = sum[0];
    if (s.flags & F_PRECOND) {
      const double rho = sum[0];
      double be = 0.0;
      if (!(rho > 0.0) || !isfinite(rho)) {
        s.status = ST_BREAKDOWN;
        return false;
      }
      if (s.k == 0) sc.first = 1;
      else be = rho / s.delta;
      s.delta = rho;
      s.beta = be;
      sc.be = be;
      return true;
    }
    if (s.flags & F_BB_PENDING) {
      s.bb = sum[1];
      s.thr = (s.tol * s.tol) * s.bb;
      s.flags &= ~F_BB_PENDING;
      if (s.bb == 0.0) {
        s.status = ST_ZERO_RHS;
        return false;
      }
    }
    const int st = stop_code(gamma, s.thr, s.k, s.maxit, s.tol);
    double be = 0.0;
    if (s.k == 0) sc.first = 1;
    else be = gamma / s.gamma;
    s.gamma = gamma;
    s.delta = gamma;  // alpha's numerator for pass 2
    s.status = st;
    if (st != ST_RUNNING) return false;
    s.beta = be;
    sc.be = be;
    return true;
  } else if constexpr (KIND == K_CG2) {
    // Algorithm 1: alpha = (r,r) / (p, A p).
    if (s.status != ST_RUNNING) return false;
    const double pi = sum[0];
    if (!(pi > 0.0) || !isfinite(pi)) {
      s.status = ST_BREAKDOWN;
      return false;
    }
    // delta holds alpha's numerator: rho = (r,z) preconditioned, else (r,r)
    // (one field read unconditionally: a select between two fields of the
    // state would make the compiler address it through scratch memory)
    s.alpha = s.delta / pi;
    s.k += 1;
    sc.al = s.alpha;
    return true;
  } else if constexpr (KIND == K_REF_SCALE) {
    // Outer refinement step: test the true FP64 residual, then scale it.
    if (s.status != ST_RUNNING) return false;
    const double g = sum[0];
    if (s.flags & F_BB_PENDING) {
      s.bb = sum[1];
      s.thr = (s.tol * s.tol) * s.bb;
      s.flags &= ~F_BB_PENDING;
      if (s.bb == 0.0) {
        s.status = ST_ZERO_RHS;
        return false;
      }
    }
    s.res2 = g;
    int st = ST_RUNNING;
    if (!isfinite(g)) st = ST_BREAKDOWN;
    else if (g <= s.thr) st = ST_OK;
    else if (s.k >= s.maxit) st = ST_NOT_CONVERGED;
    s.status = st;
    if (st != ST_RUNNING) return false;
    s.scale = sqrt(g);
    s.kin = 0;
    sc.inv = 1.0 / s.scale;
    return true;
  } else if constexpr (KIND == K_CHEBF) {
    // Preconditioned inner solve: the inner stop test on gamma = (r, r) of
    // the inner residual (the scale pass or pass 2 before this one), before
    // z = M^-1 r is formed; the threshold as in the unpreconditioned one.
    if (s.status != ST_RUNNING) return false;
    const double gamma = sum[0];
    if (s.kin == 0) {
      const double e = fmax(s.inner_tol, (0.5 * s.tol) * (sqrt(s.bb) / s.scale));
      s.gamma0 = gamma;
      s.thr_in = (e * e) * gamma;
    }
    s.gamma = gamma;
    if (!isfinite(gamma) || gamma <= s.thr_in || s.k >= s.maxit) {
      s.status = ST_INNER_DONE;
      return false;
    }
    return true;
  } else if constexpr (KIND == K_CG1F) {
    if (s.status != ST_RUNNING) return false;
    if (s.flags & F_PRECOND) {
      // the one slot is rho = (r, z) from the Chebyshev pass (which made the
      // stop test); beta = rho / rho_old with rho kept in delta, p = z + beta p
      const double rho = sum[0];
      if (!(rho > 0.0) || !isfinite(rho)) {
        s.status = ST_INNER_DONE;
        return false;
      }
      double be = 0.0;
      if (s.kin == 0) sc.first = 1;
      else be = rho / s.delta;
      s.delta = rho;
      s.beta = be;
      sc.be = be;
      return true;
    }
    const double gamma = sum[0];
    double be = 0.0;
    if (s.kin == 0) {
      // inner stop: relative residual e = max(inner_tol, (tol/2) ||b|| / s),
      // no further than the outer tolerance needs (s = ||b - A x||)
      const double e = fmax(s.inner_tol, (0.5 * s.tol) * (sqrt(s.bb) / s.scale));
      s.gamma0 = gamma;
      s.thr_in = (e * e) * gamma;
      sc.first = 1;
    } else {
      be = gamma / s.gamma;
    }
    s.gamma = gamma;
    s.delta = gamma;  // alpha's numerator for pass 2
    if (!isfinite(gamma) || gamma <= s.thr_in || s.k >= s.maxit) {
      s.status = ST_INNER_DONE;
      return false;
    }
    s.beta = be;
    sc.be = be;
    return true;
  } else if constexpr (KIND == K_CG2F) {
    if (s.status != ST_RUNNING) return false;
    const double pi = sum[0];
    if (!(pi > 0.0) || !isfinite(pi)) {
      s.status = ST_INNER_DONE;
      return false;
    }
    // delta: rho = (r, z) preconditioned, else (r, r)
    s.alpha = s.delta / pi;
    s.k += 1;
    s.kin += 1;
    sc.al = s.alpha;
    return true;
  } else if constexpr (KIND == K_REF_UPDATE) {
    if (s.status != ST_INNER_DONE) return false;
    if (s.kin == 0) {
      s.status = ST_BREAKDOWN;
      return false;
    }
    s.status = ST_RUNNING;
    s.outer += 1;
    sc.al = s.scale;
    return true;
  }
  return false;
}

template <int KIND>
constexpr int ndots_in() {  // partial slots the prologue consumes
  return (KIND == K_PCG || KIND == K_PCGX || KIND == K_INIT_W || KIND == K_CG1 ||
          KIND == K_REF_SCALE)
             ? 2
         : (KIND == K_CG2 || KIND == K_CG2X || KIND == K_CG1F || KIND == K_CG2F ||
            KIND == K_CG2FX || KIND == K_CHEBF)
             ? 1
             : 0;
}

template <int KIND>
constexpr int ndots_out() {  // partial slots the body produces
  return (KIND == K_INIT_WU || KIND == K_PPCG) ? 3
         : (KIND == K_INIT_R || KIND == K_INIT_W || KIND == K_PCG || KIND == K_PCGX ||
            KIND == K_RESID)
             ? 2
         : (KIND == K_CG1 || KIND == K_CG2 || KIND == K_CG2X || KIND == K_REF_SCALE ||
            KIND == K_CG1F || KIND == K_CG2F || KIND == K_CG2FX || KIND == K_DOT)
             ? 1
             : 0;
}

// The passes whose solution update is deferred (see cg_internal.h): FP64 CG
// (x, counted by k) and the FP32 inner solve (d, counted by kin).
template <int KIND>
constexpr bool defers_x() {
  return KIND == K_PCG || KIND == K_PCGX || KIND == K_CG1 || KIND == K_CG2 || KIND == K_CG2X ||
         KIND == K_CG1F || KIND == K_CG2F || KIND == K_CG2FX || KIND == K_CHEB ||
         KIND == K_CHEBF;
}

template <int KIND>
constexpr bool inner_kind() {
  return KIND == K_CG1F || KIND == K_CG2F || KIND == K_CG2FX || KIND == K_CHEBF;
}

// transition<KIND> plus the deferred-x bookkeeping: sc.xu when this pass ends
// an even iteration (sc.alp = the previous iteration's alpha), and `flush`
// when this pass stops a running solve whose last iteration was odd (then
// sc.alp = that iteration's alpha, whose update is still pending).
template <int KIND>
__device__ __forceinline__ bool transition_x(State& s, const double* sum, Sc& sc, bool& flush) {
  const bool was_running = s.status == ST_RUNNING;
  const double alpha_before = s.alpha;
  const bool run = transition<KIND>(s, sum, sc);
  flush = false;
  if constexpr (defers_x<KIND>()) {
    const int k = inner_kind<KIND>() ? s.kin : s.k;
    if (run && KIND != K_CG1 && KIND != K_CG1F && KIND != K_CHEB && KIND != K_CHEBF &&
        !(k & 1)) {
      sc.xu = 1;
      sc.alp = alpha_before;
    }
    if (was_running && s.status != ST_RUNNING && (k & 1)) {
      flush = true;
      sc.alp = s.alpha;
    }
  }
  return run;
}

// ------------------------------------------------------------- reductions --

// Cross-tile stage: the 256 threads of a tile group sum part[d*T + k] for
// k = tid, tid+256, ... in order, butterfly within each wavefront, then add
// the four wavefront values in order.  Every thread of the group receives
// the sums.  `lds` holds 4*D doubles for this group.
template <int D>
__device__ __forceinline__ void cross_tile_sum(const double* part, int T, double* out,
                                               double* lds) {
  const int tid = threadIdx.x & (kGroup - 1), lane = tid & (kWave - 1), wave = tid >> 6;
  double v[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    double acc = 0.0;
    for (int k = tid; k < T; k += kGroup) acc = acc + part[(size_t)d * T + k];
    v[d] = wave_sum(acc);
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) lds[wave * D + d] = v[d];
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < D; ++d) {
    double t = lds[d];
#pragma unroll
    for (int w = 1; w < kWavesPerTile; ++w) t = t + lds[w * D + d];
    out[d] = t;
  }
  __syncthreads();
}

// Per-tile partials: butterfly each lane value, add wavefronts in order, and
// let the group's first thread store part[d*T + t].  `lds` holds 2*4*D
// doubles for this group (double-buffered by `par` so one barrier suffices).
template <int D>
__device__ __forceinline__ void tile_partial(const double* lv, double* part, int T, int t,
                                             double* lds, int par) {
  const int tid = threadIdx.x & (kGroup - 1), lane = tid & (kWave - 1), wave = tid >> 6;
  double* L = lds + par * kWavesPerTile * D;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double v = wave_sum(lv[d]);
    if (lane == 0) L[wave * D + d] = v;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double s = L[d];
#pragma unroll
      for (int w = 1; w < kWavesPerTile; ++w) s = s + L[w * D + d];
      part[(size_t)d * T + t] = s;
    }
  }
}

template <int CPL>
__device__ __forceinline__ double fold(const double (&acc)[CPL]) {
  double v = acc[0];
#pragma unroll
  for (int k = 1; k < CPL; ++k) v = v + acc[k];
  return v;
}

// ------------------------------------------------------------- tile bodies --
//
// Each body handles tile t for the calling wavefront (rows s.j0..s.j1-1) and
// leaves the lane's dot-product values in lv[].  Loops are wavefront-uniform.

// Tile-edge addressing: lane 0 reads the value left of the tile, lane 63 the
// value right of it, every other lane re-reads its own first element (an L1
// hit), so the edge values come from one load of the whole wavefront with no
// divergent branch.  `emask` is set on the lanes whose edge value is inside the
// grid; elsewhere the edge reads as zero.
struct EdgeAddr {
  int off;     // column offset of this lane's edge load within a row
  bool emask;  // this lane supplies a real neighbour value
};

template <int CPL>
__device__ __forceinline__ EdgeAddr edge_addr(const Strip& s, const Geo& g) {
  EdgeAddr e;
  e.off = s.c;
  e.emask = false;
  if (s.lane == 0 && s.tx > 0) {
    e.off = s.ct - 1;
    e.emask = true;
  }
  if (s.lane == kWave - 1 && s.tx + 1 < g.ntx) {
    e.off = s.ct + kWave * CPL;
    e.emask = true;
  }
  return e;
}

// The same edge values from loads that touch two cache lines: lanes 0-31 all
// read lane 0's address, lanes 32-63 lane 63's (the tile's first column
// where there is no neighbour), so the other lanes add no lines of their own.
// Classic pass 1, which issues two edge loads a row (r and p_old), runs 4 %
// faster so at 4096^2; the passes with one edge load a row, issued beside
// the row's own load, ran slightly slower and keep edge_addr.
template <int CPL>
__device__ __forceinline__ EdgeAddr edge_addr2(const Strip& s, const Geo& g) {
  EdgeAddr e;
  const bool west = s.lane < kWave / 2;
  const bool has = west ? s.tx > 0 : s.tx + 1 < g.ntx;
  e.off = has ? (west ? s.ct - 1 : s.ct + kWave * CPL) : s.ct;
  e.emask = has && (s.lane == 0 || s.lane == kWave - 1);
  return e;
}

// Row walkers shared by every stencil body (walk, which hands the 5-point
// operators to walk2d).  For the wavefront's strip a walker
// keeps rows j-1, j, j+1 of the halo vector H and the point data of row j in
// registers, and issues the loads of halo row j+PD+1 and point row j+PD
// before it computes row j, so each wavefront keeps PD+1 rows of loads in
// flight.  Loads and arithmetic are separate stages (hload/eload load only;
// hmake/emake combine the loaded values when the row enters the window), and
// every prefetch load is unconditional: a row outside the grid or past the
// strip's north halo is replaced by a valid row whose value is then ignored.
// That keeps the number of loads in flight static, so the compiler waits only
// for the row it is about to use.
//   hload(off) -> raw halo data of the row at offset `off`
//   hmake(raw) -> Row: H at this lane's columns
//   eload(off) -> raw tile-edge data of that row (one load per vector)
//   emake(raw) -> H just outside the tile for lanes 0 / 63 (zero elsewhere)
//   point(off) -> Bundle: the point-wise operands of that row
//   comp(off, S, C, N, W, E, bundle): row j's arithmetic and stores
//
// D3 (the 7-point operator of an nx x g.plane x nz grid stored as g.ny =
// g.plane * nz rows of nx): the walker marches along z instead (walk below)
// and hands comp the rows below / above too; in 2D those are zero rows.
//   comp(off, S, C, N, W, E, below, above, kc, bundle)
//
// OP selects the operator: 0 the 5-point stencil, 1 the 7-point one (D3
// above), 2 the variable-coefficient 5-point one, for which the walker also
// loads the row's four face conductivities (kc: Kc rows of the west, east,
// south and north arrays that g.kc holds one after the other, each laid out
// like a vector) PD rows ahead with the point data.
//
// The walker of the 5-point operators (OP 0, and OP 2 with the row's four
// face conductivities loaded with the point data).  With g.alt the odd
// wavefronts of a tile walk their strip from its last row up (S and N keep
// their meaning: comp still gets rows j-1, j, j+1), so that the row between
// two wavefronts' strips is loaded by both at about the same time: the
// second load is a cache hit, where top-down walks put those two loads a
// whole strip apart.  DYN: up is the caller's (a wavefront-uniform flag);
// else always top down, with the address arithmetic of a plain forward walk.
template <bool DYN, typename T, int CPL, int PD, int OP, class HLoad, class HMake, class ELoad,
          class EMake, class Point, class Comp>
__device__ __forceinline__ void walk2d_dir(const Geo& g, const Strip& s, HLoad hload,
                                           HMake hmake, ELoad eload, EMake emake, Point point,
                                           Comp comp, bool up_arg) {
  static_assert(OP == 0 || OP == 2, "5-point operators only");
  using R = Row<T, CPL>;
  using RawH = decltype(hload((size_t)0));
  using RawE = decltype(eload((size_t)0));
  using B = decltype(point((size_t)0));
  const size_t P = g.pitch;
  const bool up = DYN ? up_arg : false;
  const int dir = up ? -1 : 1;
  const int jst = up ? s.j1 - 1 : s.j0;  // first row walked
  const int jen = up ? s.j0 - 1 : s.j1;  // one past the last, in walk order
  // halo rows ahead of the walk: down to row j0 - 1 walking up, up to row j1
  // walking down (when inside the grid); loads of rows past them re-read the
  // last one, whose value is then ignored
  const int hlim = up ? max(s.j0 - 1, 0) : min(s.j1, g.ny - 1);
  auto ahead_ok = [&](int r) { return up ? (r >= s.j0 - 1 && r >= 0) : r <= hlim; };
  auto ahead_row = [&](int r) { return up ? max(r, hlim) : min(r, hlim); };
  // point rows ahead of the walk, clamped to the strip's far end
  auto point_row = [&](int r) { return up ? max(r, s.j0) : min(r, s.j1 - 1); };
  using K = Kc<T, CPL>;
  const size_t kst = (size_t)g.kcs;  // from one coefficient array to the next
  auto kload = [&](size_t off) {
    K k;
    if constexpr (OP == 2) {
      const double* c0 = g.kc + off + s.c;
      k.w = ldrow<T, CPL>(c0);
      k.e = ldrow<T, CPL>(c0 + kst);
      k.s = ldrow<T, CPL>(c0 + 2 * kst);
      k.n = ldrow<T, CPL>(c0 + 3 * kst);
    }
    return k;
  };
  K qk[OP == 2 ? PD : 1];
  R hB = zrow<T, CPL>();  // the row behind the walk (row jst - dir)
  {
    const int rb = jst - dir;
    const int rbl = up ? min(rb, g.ny - 1) : max(rb, 0);
    const R v = hmake(hload((size_t)rbl * P));
    if (up ? rb < g.ny : rb >= 0) hB = v;
  }
  R hC = hmake(hload((size_t)jst * P));
  T eC = emake(eload((size_t)jst * P));
  RawH q[PD];   // raw halo rows jst + dir, ..., jst + PD dir
  RawE qe[PD];
  bool qv[PD];  // the row exists (inside the grid, not past the strip's halo)
  B pt[PD];     // point data of rows jst .. jst + (PD - 1) dir
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    const int r = jst + dir * (1 + k);
    qv[k] = ahead_ok(r);
    const size_t ro = (size_t)ahead_row(r) * P;
    q[k] = hload(ro);
    qe[k] = eload(ro);
    pt[k] = point((size_t)point_row(jst + dir * k) * P);
    if constexpr (OP == 2) qk[k] = kload((size_t)point_row(jst + dir * k) * P);
  }
  for (int j = jst; j != jen; j += dir) {
    const size_t o = (size_t)j * P;
    // loads of the rows needed PD steps from now
    const int rh = j + dir * (PD + 1);
    const bool nv = ahead_ok(rh);
    const size_t ho = (size_t)ahead_row(rh) * P;
    const RawH hn = hload(ho);
    const RawE en = eload(ho);
    const B pn = point((size_t)point_row(j + dir * PD) * P);
    K kn;
    if constexpr (OP == 2) kn = kload((size_t)point_row(j + dir * PD) * P);
    // row j + dir enters the window
    R hA = hmake(q[0]);
    T eA = emake(qe[0]);
    if (!qv[0]) {
      hA = zrow<T, CPL>();
      eA = T(0);
    }
    R W, E;
    west_east<T, CPL>(hC, eC, eC, W, E);
    const R zr = zrow<T, CPL>();
    // S is row j - 1 and N row j + 1 in either direction
    if (up) comp(o, hA, hC, hB, W, E, zr, zr, qk[0], pt[0]);
    else comp(o, hB, hC, hA, W, E, zr, zr, qk[0], pt[0]);
    hB = hC;
    hC = hA;
    eC = eA;
#pragma unroll
    for (int k = 0; k + 1 < PD; ++k) {
      q[k] = q[k + 1];
      qe[k] = qe[k + 1];
      qv[k] = qv[k + 1];
      pt[k] = pt[k + 1];
      if constexpr (OP == 2) qk[k] = qk[k + 1];
    }
    q[PD - 1] = hn;
    qe[PD - 1] = en;
    qv[PD - 1] = nv;
    pt[PD - 1] = pn;
    if constexpr (OP == 2) qk[PD - 1] = kn;
  }
}

// ALT = false: always top down (the passes of pipelined solves, whose plans
// never set g.alt, and the apply pass, which sums nothing).  One loop serves
// both directions: measured faster than a loop per direction (stencil_dot
// 81.7 against 82.9 us at 4096^2, update_norm 141.2 against 144.7 us).
template <typename T, int CPL, int PD, int OP, bool ALT, class HLoad, class HMake, class ELoad,
          class EMake, class Point, class Comp>
__device__ __forceinline__ void walk2d(const Geo& g, const Strip& s, HLoad hload, HMake hmake,
                                       ELoad eload, EMake emake, Point point, Comp comp) {
  if (s.j0 >= s.j1) return;
  walk2d_dir<ALT, T, CPL, PD, OP>(g, s, hload, hmake, eload, emake, point, comp,
                                  ALT && g.alt && (s.wave & 1));
}

// The 7-point walker's in-plane neighbours, rows y - 1 and y + 1 of the plane
// a wavefront is at, are the rows the tile's other wavefronts hold at the
// same step: each wavefront publishes its row in an LDS exchange buffer and,
// after one barrier per plane, reads its two neighbours.  The tile's outer
// rows y0 - 1 and y0 + 4 come from loads, in one of three forms:
//   ZX_EDGE  wavefronts 0 and 3 load them whole (zwalk_xch);
//   ZX_HALF  every wavefront loads half of one, one value per lane
//            (zwalk_half, halo vectors stored as is);
//   classic pass 1, whose halo vector is formed from two vectors, splits
//   them one vector row per wavefront (zwalk_split).
// Measured at 256^3 (HIP events): ZX_HALF for the passes with one halo
// vector (update_norm_nx 78.5 -> 73.3 us, pcg_pass 279.2 -> 277.7 us against
// every wavefront loading a whole outer row), except the odd pipelined pass,
// which runs 0.7 % faster with ZX_EDGE; zwalk_split took classic pass 1 from
// 86.2 to 79.6 us (rocprofv3) against ZX_EDGE.  Loading the neighbour rows
// in each wavefront instead of any exchange ran classic pass 1 at 108.0 us.
constexpr int ZX_EDGE = 1, ZX_HALF = 2;

// The exchange rows: two buffers (alternate planes) of six rows (the tile's
// outer row y0 - 1, its four rows, its outer row y0 + 4) of one FP64 pair per
// lane.
__shared__ __align__(16) double zm_x[2 * (kWavesPerTile + 2) * kWave * 2];

__device__ __forceinline__ void zm_store(double* xb, int slot, int lane, const Row<double, 2>& v) {
  *reinterpret_cast<double2*>(xb + (slot * kWave + lane) * 2) = make_double2(v.e[0], v.e[1]);
}

__device__ __forceinline__ Row<double, 2> zm_load(const double* xb, int slot, int lane) {
  const double2 d = *reinterpret_cast<const double2*>(xb + (slot * kWave + lane) * 2);
  Row<double, 2> v;
  v.e[0] = d.x;
  v.e[1] = d.y;
  return v;
}

// The z-march with the exchange, the outer rows loaded by wavefronts 0 and 3
// (ZX_EDGE).  After one barrier per plane every wavefront reads its two
// neighbours (zero outside the plane).  A wavefront whose row lies past the plane still takes every
// step (its loads read a valid row, its exchange row is zero, it computes
// nothing), so the four wavefronts pass the same barriers.
template <typename T, int CPL, int PD, class HLoad, class HMake, class ELoad, class EMake,
          class Point, class Comp>
__device__ __forceinline__ void zwalk_xch(const Geo& g, const Strip& s, HLoad hload, HMake hmake,
                                          ELoad eload, EMake emake, Point point, Comp comp) {
  static_assert(sizeof(T) == 8 && CPL == 2, "the 3D walker exchanges FP64 pairs");
  using R = Row<T, CPL>;
  using RawH = decltype(hload((size_t)0));
  using RawE = decltype(eload((size_t)0));
  using B = decltype(point((size_t)0));
  const size_t P = g.pitch;
  const int pl = g.plane, nz = g.ny / pl;
  const int w = __builtin_amdgcn_readfirstlane(s.wave);
  const int z0 = s.z0, z1 = s.z1;
  const bool live = s.y < pl;
  const int y = live ? s.y : pl - 1;
  auto off = [&](int z, int yy) { return ((size_t)z * pl + yy) * P; };
  // the outer row this wavefront forms: y0 - 1 (wavefront 0), y0 + 4 (3)
  const bool outer = w == 0 || w == kWavesPerTile - 1;
  const int yo = (w == 0) ? s.y - 1 : s.y + 1;
  const bool has_o = outer && yo >= 0 && yo < pl;
  const int yoc = has_o ? yo : y;
  const int oslot = (w == 0) ? 0 : kWavesPerTile + 1;
  const int zmax = min(z1, nz - 1);  // last plane worth loading ahead
  const Kc<T, CPL> kz{};
  const R zr = zrow<T, CPL>();
  __syncthreads();  // every wavefront has read the previous tile's exchange rows
  R hB = zr;  // plane z - 1
  {
    const R v = hmake(hload(off(max(z0 - 1, 0), y)));
    if (z0 > 0) hB = v;
  }
  R hC = hmake(hload(off(z0, y)));
  T eC = emake(eload(off(z0, y)));
  RawH q[PD];   // raw row y of planes z+1 .. z+PD
  RawE qe[PD];
  bool qv[PD];  // the plane exists (inside the grid, not past the tile's halo)
  B pt[PD];     // point data of planes z .. z+PD-1
  RawH qo[PD];  // the outer row of planes z .. z+PD-1 (wavefronts 0 and 3)
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    const int zr1 = z0 + 1 + k;
    qv[k] = zr1 <= zmax;
    const size_t ro = off(min(zr1, zmax), y);
    q[k] = hload(ro);
    qe[k] = eload(ro);
    const int zp = min(z0 + k, z1 - 1);
    pt[k] = point(off(zp, y));
    qo[k] = q[k];  // (unused off the outer wavefronts)
    if (outer) qo[k] = hload(off(zp, yoc));
  }
  for (int z = z0; z < z1; ++z) {
    const size_t o = off(z, y);
    // loads of the planes needed PD steps from now
    const int zh = z + PD + 1;
    const bool nv = zh <= zmax;
    const size_t ho = off(min(zh, zmax), y);
    const RawH hn = hload(ho);
    const RawE en = eload(ho);
    const int zp = min(z + PD, z1 - 1);
    const B pn = point(off(zp, y));
    RawH on = hn;
    if (outer) on = hload(off(zp, yoc));
    // this plane's rows into the exchange buffer
    double* xb = zm_x + ((z - z0) & 1) * ((kWavesPerTile + 2) * kWave * 2);
    zm_store(xb, w + 1, s.lane, live ? hC : zr);
    if (outer) zm_store(xb, oslot, s.lane, has_o ? hmake(qo[0]) : zr);
    // plane z + 1 enters the window
    R hA = hmake(q[0]);
    T eA = emake(qe[0]);
    if (!qv[0]) {
      hA = zr;
      eA = T(0);
    }
    R W, E;
    west_east<T, CPL>(hC, eC, eC, W, E);
    __syncthreads();
    const R Sr = zm_load(xb, w, s.lane);
    const R Nr = zm_load(xb, w + 2, s.lane);
    if (live) comp(o, Sr, hC, Nr, W, E, hB, hA, kz, pt[0]);
    hB = hC;
    hC = hA;
    eC = eA;
#pragma unroll
    for (int k = 0; k + 1 < PD; ++k) {
      q[k] = q[k + 1];
      qe[k] = qe[k + 1];
      qv[k] = qv[k + 1];
      pt[k] = pt[k + 1];
      qo[k] = qo[k + 1];
    }
    q[PD - 1] = hn;
    qe[PD - 1] = en;
    qv[PD - 1] = nv;
    pt[PD - 1] = pn;
    qo[PD - 1] = on;
  }
}

// The raw halves of the tile's outer rows for zwalk_split: two buffers of
// four rows (row y0 - 1's first and second vector, then row y0 + 4's).
__shared__ __align__(16) double zm_r[2 * 4 * kWave * 2];

// The z-march of a pass whose halo vector is formed from two vectors (classic
// pass 1: p = r + beta p_old).  As zwalk_xch, but the tile's two outer rows
// cost four row loads, one per wavefront: wavefront w loads vector w & 1 of
// row y0 - 1 (w < 2) or y0 + 4 (w >= 2) and publishes it raw; after the
// barrier wavefront 0 joins row y0 - 1's halves into its south neighbour and
// wavefront 3 row y0 + 4's into its north one, with the same arithmetic as
// hmake.  Every wavefront then issues three row loads a plane (against four
// for wavefronts 0 and 3 and two for 1 and 2 in zwalk_xch).
//   hpart(off, k) -> Row: vector k of the halo sources at offset off
//   hjoin(a, b)   -> Row: hmake of the raw pair (a, b)
template <typename T, int CPL, int PD, class HLoad, class HMake, class HPart, class HJoin,
          class ELoad, class EMake, class Point, class Comp>
__device__ __forceinline__ void zwalk_split(const Geo& g, const Strip& s, HLoad hload,
                                            HMake hmake, HPart hpart, HJoin hjoin, ELoad eload,
                                            EMake emake, Point point, Comp comp) {
  static_assert(sizeof(T) == 8 && CPL == 2, "the 3D walker exchanges FP64 pairs");
  using R = Row<T, CPL>;
  using RawH = decltype(hload((size_t)0));
  using RawE = decltype(eload((size_t)0));
  using B = decltype(point((size_t)0));
  const size_t P = g.pitch;
  const int pl = g.plane, nz = g.ny / pl;
  const int w = __builtin_amdgcn_readfirstlane(s.wave);
  const int z0 = s.z0, z1 = s.z1;
  const bool live = s.y < pl;
  const int y = live ? s.y : pl - 1;
  const int y0 = s.y - w;  // the tile's first in-plane row
  auto off = [&](int z, int yy) { return ((size_t)z * pl + yy) * P; };
  // the outer half this wavefront loads (a row outside the plane is replaced
  // by row y, whose value is then ignored)
  const int yo = (w < 2) ? y0 - 1 : y0 + kWavesPerTile;
  const int yoc = (yo >= 0 && yo < pl) ? yo : y;
  const int part = w & 1;
  const bool has_s = y0 > 0, has_n = y0 + kWavesPerTile < pl;  // for wavefronts 0 / 3
  const int zmax = min(z1, nz - 1);  // last plane worth loading ahead
  const Kc<T, CPL> kz{};
  const R zr = zrow<T, CPL>();
  __syncthreads();  // every wavefront has read the previous tile's exchange rows
  R hB = zr;  // plane z - 1
  {
    const R v = hmake(hload(off(max(z0 - 1, 0), y)));
    if (z0 > 0) hB = v;
  }
  R hC = hmake(hload(off(z0, y)));
  T eC = emake(eload(off(z0, y)));
  RawH q[PD];   // raw row y of planes z+1 .. z+PD
  RawE qe[PD];
  bool qv[PD];  // the plane exists (inside the grid, not past the tile's halo)
  B pt[PD];     // point data of planes z .. z+PD-1
  R qo[PD];     // this wavefront's outer half of planes z .. z+PD-1
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    const int zr1 = z0 + 1 + k;
    qv[k] = zr1 <= zmax;
    const size_t ro = off(min(zr1, zmax), y);
    q[k] = hload(ro);
    qe[k] = eload(ro);
    const int zp = min(z0 + k, z1 - 1);
    pt[k] = point(off(zp, y));
    qo[k] = hpart(off(zp, yoc), part);
  }
  for (int z = z0; z < z1; ++z) {
    const size_t o = off(z, y);
    // loads of the planes needed PD steps from now
    const int zh = z + PD + 1;
    const bool nv = zh <= zmax;
    const size_t ho = off(min(zh, zmax), y);
    const RawH hn = hload(ho);
    const RawE en = eload(ho);
    const int zp = min(z + PD, z1 - 1);
    const B pn = point(off(zp, y));
    const R on = hpart(off(zp, yoc), part);
    // this plane's rows and outer halves into the exchange buffers
    const int b = (z - z0) & 1;
    double* xb = zm_x + b * ((kWavesPerTile + 2) * kWave * 2);
    double* rb = zm_r + b * (4 * kWave * 2);
    zm_store(xb, w + 1, s.lane, live ? hC : zr);
    zm_store(rb, w, s.lane, qo[0]);
    // plane z + 1 enters the window
    R hA = hmake(q[0]);
    T eA = emake(qe[0]);
    if (!qv[0]) {
      hA = zr;
      eA = T(0);
    }
    R W, E;
    west_east<T, CPL>(hC, eC, eC, W, E);
    __syncthreads();
    R Sr, Nr;
    if (w == 0) Sr = has_s ? hjoin(zm_load(rb, 0, s.lane), zm_load(rb, 1, s.lane)) : zr;
    else Sr = zm_load(xb, w, s.lane);
    if (w == kWavesPerTile - 1) Nr = has_n ? hjoin(zm_load(rb, 2, s.lane), zm_load(rb, 3, s.lane)) : zr;
    else Nr = zm_load(xb, w + 2, s.lane);
    if (live) comp(o, Sr, hC, Nr, W, E, hB, hA, kz, pt[0]);
    hB = hC;
    hC = hA;
    eC = eA;
#pragma unroll
    for (int k = 0; k + 1 < PD; ++k) {
      q[k] = q[k + 1];
      qe[k] = qe[k + 1];
      qv[k] = qv[k + 1];
      pt[k] = pt[k + 1];
      qo[k] = qo[k + 1];
    }
    q[PD - 1] = hn;
    qe[PD - 1] = en;
    qv[PD - 1] = nv;
    pt[PD - 1] = pn;
    qo[PD - 1] = on;
  }
}

// The tile's two outer rows for zwalk_half: two buffers of two rows of the
// tile's 2 * kWave columns, in column order.
__shared__ __align__(16) double zm_h[2 * 2 * 2 * kWave];

// The z-march of a pass whose halo vector is stored as is (V).  As
// zwalk_xch, but the tile's two outer rows cost one half-row load per
// wavefront: wavefront w loads columns [64 (w & 1), 64 (w & 1) + 64) of the
// tile's row y0 - 1 (w < 2) or y0 + 4 (w >= 2), one value per lane, into an
// LDS row buffer; after the barrier wavefronts 0 and 3 read their outer
// neighbour from it.  Every wavefront issues the same loads, with no branch.
template <typename T, int CPL, int PD, class HLoad, class ELoad, class EMake, class Point,
          class Comp>
__device__ __forceinline__ void zwalk_half(const Geo& g, const Strip& s, const T* V, HLoad hload,
                                           ELoad eload, EMake emake, Point point, Comp comp) {
  static_assert(sizeof(T) == 8 && CPL == 2, "the 3D walker exchanges FP64 pairs");
  using R = Row<T, CPL>;
  using RawE = decltype(eload((size_t)0));
  using B = decltype(point((size_t)0));
  const size_t P = g.pitch;
  const int pl = g.plane, nz = g.ny / pl;
  const int w = __builtin_amdgcn_readfirstlane(s.wave);
  const int z0 = s.z0, z1 = s.z1;
  const bool live = s.y < pl;
  const int y = live ? s.y : pl - 1;
  const int y0 = s.y - w;  // the tile's first in-plane row
  auto off = [&](int z, int yy) { return ((size_t)z * pl + yy) * P; };
  // this lane's outer value: a column of the padded row (a row outside the
  // plane is replaced by row y, whose value is then ignored)
  const int yo = (w < 2) ? y0 - 1 : y0 + kWavesPerTile;
  const int yoc = (yo >= 0 && yo < pl) ? yo : y;
  const int hcol = s.ct + (w & 1) * kWave + s.lane;
  const int hslot = (w >> 1) * (2 * kWave) + (w & 1) * kWave + s.lane;
  const bool has_s = y0 > 0, has_n = y0 + kWavesPerTile < pl;  // for wavefronts 0 / 3
  const int zmax = min(z1, nz - 1);  // last plane worth loading ahead
  const Kc<T, CPL> kz{};
  const R zr = zrow<T, CPL>();
  __syncthreads();  // every wavefront has read the previous tile's exchange rows
  R hB = zr;  // plane z - 1
  {
    const R v = hload(off(max(z0 - 1, 0), y));
    if (z0 > 0) hB = v;
  }
  R hC = hload(off(z0, y));
  T eC = emake(eload(off(z0, y)));
  R q[PD];      // row y of planes z+1 .. z+PD
  RawE qe[PD];
  bool qv[PD];  // the plane exists (inside the grid, not past the tile's halo)
  B pt[PD];     // point data of planes z .. z+PD-1
  T qo[PD];     // this lane's outer value of planes z .. z+PD-1
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    const int zr1 = z0 + 1 + k;
    qv[k] = zr1 <= zmax;
    const size_t ro = off(min(zr1, zmax), y);
    q[k] = hload(ro);
    qe[k] = eload(ro);
    const int zp = min(z0 + k, z1 - 1);
    pt[k] = point(off(zp, y));
    qo[k] = V[off(zp, yoc) + hcol];
  }
  for (int z = z0; z < z1; ++z) {
    const size_t o = off(z, y);
    // loads of the planes needed PD steps from now
    const int zh = z + PD + 1;
    const bool nv = zh <= zmax;
    const size_t ho = off(min(zh, zmax), y);
    const R hn = hload(ho);
    const RawE en = eload(ho);
    const int zp = min(z + PD, z1 - 1);
    const B pn = point(off(zp, y));
    const T on = V[off(zp, yoc) + hcol];
    // this plane's rows and outer values into the exchange buffers
    const int b = (z - z0) & 1;
    double* xb = zm_x + b * ((kWavesPerTile + 2) * kWave * 2);
    double* hb = zm_h + b * (2 * 2 * kWave);
    zm_store(xb, w + 1, s.lane, live ? hC : zr);
    hb[hslot] = qo[0];
    // plane z + 1 enters the window
    R hA = q[0];
    T eA = emake(qe[0]);
    if (!qv[0]) {
      hA = zr;
      eA = T(0);
    }
    R W, E;
    west_east<T, CPL>(hC, eC, eC, W, E);
    __syncthreads();
    R Sr, Nr;
    if (w == 0) Sr = has_s ? zm_load(hb, 0, s.lane) : zr;
    else Sr = zm_load(xb, w, s.lane);
    if (w == kWavesPerTile - 1) Nr = has_n ? zm_load(hb, 1, s.lane) : zr;
    else Nr = zm_load(xb, w + 2, s.lane);
    if (live) comp(o, Sr, hC, Nr, W, E, hB, hA, kz, pt[0]);
    hB = hC;
    hC = hA;
    eC = eA;
#pragma unroll
    for (int k = 0; k + 1 < PD; ++k) {
      q[k] = q[k + 1];
      qe[k] = qe[k + 1];
      qv[k] = qv[k + 1];
      pt[k] = pt[k + 1];
      qo[k] = qo[k + 1];
    }
    q[PD - 1] = hn;
    qe[PD - 1] = en;
    qv[PD - 1] = nv;
    pt[PD - 1] = pn;
    qo[PD - 1] = on;
  }
}

// The entry point of every body, and the 7-point operator's walker: the
// z-march (strip_of: the wavefront owns in-plane row y and walks it through
// the tile's planes).  Plane z - 1 (behind), z and z + 1 (ahead) of row y are
// the window, as rows j - 1, j, j + 1 are in 2D (ZX_EDGE outer-row loads;
// walk_plain takes zwalk_half, classic pass 1 zwalk_split).  comp gets S / N = rows y -/+ 1 (zero outside the
// plane) and below / above = planes z -/+ 1 (zero outside the grid).
template <typename T, int CPL, int PD, int OP, bool ALT = true, int ZX = ZX_EDGE, class HLoad,
          class HMake, class ELoad, class EMake, class Point, class Comp>
__device__ __forceinline__ void walk(const Geo& g, const Strip& s, HLoad hload, HMake hmake,
                                     ELoad eload, EMake emake, Point point, Comp comp) {
  static_assert(OP != 1 || ZX == ZX_EDGE, "ZX_HALF is walk_plain's (it needs the halo vector)");
  if constexpr (OP != 1)
    walk2d<T, CPL, PD, OP, ALT>(g, s, hload, hmake, eload, emake, point, comp);
  else
    zwalk_xch<T, CPL, PD>(g, s, hload, hmake, eload, emake, point, comp);
}

#ifndef CG1_PREFETCH
#define CG1_PREFETCH 1
#endif

#ifndef WALK_PREFETCH
#define WALK_PREFETCH 1
#endif
#ifndef EDGE_MASKED
#define EDGE_MASKED 0
#endif

// Loaders for a halo vector that is stored as is.
template <typename T, int CPL, int OP, bool ALT = true, int ZX = ZX_HALF, class Point, class Comp>
__device__ __forceinline__ void walk_plain(const Geo& g, const Strip& s, const T* V, Point point,
                                           Comp comp) {
  const EdgeAddr ea = edge_addr<CPL>(s, g);
  const int c = s.c;
#if EDGE_MASKED
  walk<T, CPL, WALK_PREFETCH, OP, ALT, ZX>(
      g, s, [=](size_t off) { return ldrow<T, CPL>(V + off + c); },
      [](const Row<T, CPL>& r) { return r; },
      [=](size_t off) {
        T v = T(0);
        if (ea.emask) v = V[off + ea.off];
        return v;
      },
      [=](T v) { return v; }, point, comp);
#else
  if constexpr (OP == 1 && ZX == ZX_HALF) {
    zwalk_half<T, CPL, WALK_PREFETCH>(
        g, s, V, [=](size_t off) { return ldrow<T, CPL>(V + off + c); },
        [=](size_t off) { return V[off + ea.off]; }, [=](T v) { return ea.emask ? v : T(0); },
        point, comp);
  } else {
    walk<T, CPL, WALK_PREFETCH, OP, ALT, ZX>(
        g, s, [=](size_t off) { return ldrow<T, CPL>(V + off + c); },
        [](const Row<T, CPL>& r) { return r; }, [=](size_t off) { return V[off + ea.off]; },
        [=](T v) { return ea.emask ? v : T(0); }, point, comp);
  }
#endif
}

struct Empty {};

// --- K_INIT_R: r = b - A x; slots (r,r), (b,b)
// --- K_RESID:  t = b - A x; slots (t,t), (b,b)   (no store)
template <int CPL, bool STORE, int OP = 0>
__device__ __forceinline__ void body_residual(const PassArgs& a, int t, double* lv) {
  using R = Row<double, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  double a0[CPL], a1[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = a1[k] = 0.0;
  const int valid = g.nx - s.c;
  const double* B = a.b;
  double* Rr = a.r;
  walk_plain<double, CPL, OP>(
      g, s, a.x, [=](size_t off) { return ldrow<double, CPL>(B + off + s.c); },
      [&](size_t off, const R& hS, const R& hC, const R& hN, const R& W, const R& E,
          const R& B3, const R& T3, const auto& kc,
          const R& bb) {
        R res;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          res.e[k] = bb.e[k] - op_at<OP>(hS, hC, hN, W, E, B3, T3, kc, k);
          if (k < valid) {
            a0[k] = fma(res.e[k], res.e[k], a0[k]);
            a1[k] = fma(bb.e[k], bb.e[k], a1[k]);
          }
        }
        if constexpr (STORE) strow<double, CPL>(Rr + off + s.c, res, valid);
      });
  lv[0] = fold<CPL>(a0);
  lv[1] = fold<CPL>(a1);
}

// --- K_INIT_W: w = A r; slots (r,r), (w,r)
// --- K_APPLY:  y = A u; no slots
template <int CPL, bool INITW, int OP = 0>
__device__ __forceinline__ void body_apply(const PassArgs& a, int t, double* lv) {
  using R = Row<double, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  const double* U = INITW ? a.r : a.u;
  double* Y = INITW ? a.w_out : a.y;
  double a0[CPL], a1[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = a1[k] = 0.0;
  const int valid = g.nx - s.c;
  walk_plain<double, CPL, OP, false>(
      g, s, U, [](size_t) { return Empty{}; },
      [&](size_t off, const R& hS, const R& hC, const R& hN, const R& W, const R& E,
          const R& B3, const R& T3, const auto& kc,
          const Empty&) {
        R out;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          out.e[k] = op_at<OP>(hS, hC, hN, W, E, B3, T3, kc, k);
          if (INITW && k < valid) {
            a0[k] = fma(hC.e[k], hC.e[k], a0[k]);
            a1[k] = fma(out.e[k], hC.e[k], a1[k]);
          }
        }
        strow<double, CPL>(Y + off + s.c, out, valid);
      });
  lv[0] = fold<CPL>(a0);
  lv[1] = fold<CPL>(a1);
}

// --- K_DOT: slot (u, y)
template <int CPL>
__device__ __forceinline__ void body_dot(const PassArgs& a, int t, double* lv) {
  using R = Row<double, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  double a0[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = 0.0;
  const int valid = g.nx - s.c;
  // rows in the order the stencil passes of the geometry walk them (g.alt:
  // the odd wavefronts bottom up), so the sums follow the same tile order
  const bool up = g.alt && (s.wave & 1);
  for (int i = s.j0; i < s.j1; i += s.js) {
    const int j = up ? s.j1 - 1 - (i - s.j0) : i;
    const size_t o = (size_t)j * g.pitch + s.c;
    const R u = ldrow<double, CPL>(a.u + o), y = ldrow<double, CPL>(a.y + o);
#pragma unroll
    for (int k = 0; k < CPL; ++k)
      if (k < valid) a0[k] = fma(u.e[k], y.e[k], a0[k]);
  }
  lv[0] = fold<CPL>(a0);
}

// --- K_PCG: one fused iteration of Algorithm 2 (its loop body):
//   nvec = A w; z = nvec + beta z; q = w + beta q; p = r + beta p;
//   x += alpha p; r -= alpha q; w' = w - alpha z;  slots (r',r'), (w',r').
// On the first iteration z, q, p are taken as zero (z = nvec, q = w, p = r).
template <int CPL>
struct PcgRow {
  Row<double, CPL> x, r, z, q, p;
};

template <int CPL, bool XU, int OP = 0>
__device__ __forceinline__ void body_pcg(const PassArgs& a, int t, const Sc& sc, double* lv) {
  using R = Row<double, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  const double al = sc.al, be = sc.be, nal = -sc.al, alp = sc.alp;
  const bool first = sc.first;
  double a0[CPL], a1[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = a1[k] = 0.0;
  const int valid = g.nx - s.c;
  double *X = a.x, *Rv = a.r, *Z = a.z, *Q = a.q, *Pp = a.p, *Wo = a.w_out;
  walk_plain<double, CPL, OP, false, XU ? ZX_HALF : ZX_EDGE>(
      g, s, a.w_in,
      [=](size_t off) {
        PcgRow<CPL> v;
        const size_t oc = off + s.c;
        if constexpr (XU) v.x = ldrow<double, CPL>(X + oc);
        v.r = ldrow<double, CPL>(Rv + oc);
        // z, q, p are ignored on the first iteration (taken as zero)
        v.z = ldrow<double, CPL>(Z + oc);
        v.q = ldrow<double, CPL>(Q + oc);
        v.p = ldrow<double, CPL>(Pp + oc);
        return v;
      },
      [&](size_t off, const R& hS, const R& hC, const R& hN, const R& W, const R& E,
          const R& B3, const R& T3, const auto& kc,
          const PcgRow<CPL>& in) {
        R x = in.x, r = in.r, z, q, p, wo;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          const double nv = op_at<OP>(hS, hC, hN, W, E, B3, T3, kc, k);
          if (first) {
            z.e[k] = nv;
            q.e[k] = hC.e[k];
            p.e[k] = r.e[k];
          } else {
            z.e[k] = fma(be, in.z.e[k], nv);
            q.e[k] = fma(be, in.q.e[k], hC.e[k]);
            p.e[k] = fma(be, in.p.e[k], r.e[k]);
          }
          // the previous iteration's update, then this one's (never on the
          // first iteration, which is odd)
          if constexpr (XU) x.e[k] = fma(al, p.e[k], fma(alp, in.p.e[k], x.e[k]));
          r.e[k] = fma(nal, q.e[k], r.e[k]);
          wo.e[k] = fma(nal, z.e[k], hC.e[k]);
          if (k < valid) {
            a0[k] = fma(r.e[k], r.e[k], a0[k]);
            a1[k] = fma(wo.e[k], r.e[k], a1[k]);
          }
        }
        const size_t oc = off + s.c;
        strow<double, CPL>(Z + oc, z, valid);
        strow<double, CPL>(Q + oc, q, valid);
        strow<double, CPL>(Pp + oc, p, valid);
        if constexpr (XU) strow<double, CPL>(X + oc, x, valid);
        strow<double, CPL>(Rv + oc, r, valid);
        strow<double, CPL>(Wo + oc, wo, valid);
      });
  lv[0] = fold<CPL>(a0);
  lv[1] = fold<CPL>(a1);
}

// --- K_INIT_WU: w = A u; slots (r,u), (w,u), (r,r)   [preconditioned pipelined]
template <int CPL, int OP = 0>
__device__ __forceinline__ void body_init_wu(const PassArgs& a, int t, double* lv) {
  using R = Row<double, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  double a0[CPL], a1[CPL], a2[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = a1[k] = a2[k] = 0.0;
  const int valid = g.nx - s.c;
  const double* Rv = a.r;
  double* Wv = a.wv;
  walk_plain<double, CPL, OP, false>(
      g, s, a.uu, [=](size_t off) { return ldrow<double, CPL>(Rv + off + s.c); },
      [&](size_t off, const R& hS, const R& hC, const R& hN, const R& W, const R& E,
          const R& B3, const R& T3, const auto& kc,
          const R& r) {
        R out;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          out.e[k] = op_at<OP>(hS, hC, hN, W, E, B3, T3, kc, k);
          if (k < valid) {
            a0[k] = fma(r.e[k], hC.e[k], a0[k]);
            a1[k] = fma(out.e[k], hC.e[k], a1[k]);
            a2[k] = fma(r.e[k], r.e[k], a2[k]);
          }
        }
        strow<double, CPL>(Wv + off + s.c, out, valid);
      });
  lv[0] = fold<CPL>(a0);
  lv[1] = fold<CPL>(a1);
  lv[2] = fold<CPL>(a2);
}

// --- K_PPCG: one fused iteration of preconditioned pipelined CG (Ghysels and
//     Vanroose): n = A m; z = n + beta z; q = m + beta q; s = w + beta s;
//     p = u + beta p; x += alpha p; r -= alpha s; u -= alpha q;
//     w -= alpha z; slots (r,u), (w,u), (r,r) of the new vectors.  On the
//     first iteration z, q, s, p are taken as zero.
template <int CPL>
struct PpcgRow {
  Row<double, CPL> x, r, u, w, z, q, s, p;
};

template <int CPL, int OP = 0>
__device__ __forceinline__ void body_ppcg(const PassArgs& a, int t, const Sc& sc, double* lv) {
  using R = Row<double, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  const double al = sc.al, be = sc.be, nal = -sc.al;
  const bool first = sc.first;
  double a0[CPL], a1[CPL], a2[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = a1[k] = a2[k] = 0.0;
  const int valid = g.nx - s.c;
  double *X = a.x, *Rv = a.r, *U = a.uu, *Wv = a.wv, *Z = a.z, *Q = a.q, *Sv = a.sv, *Pp = a.p;
  walk_plain<double, CPL, OP, false>(
      g, s, a.mv,
      [=](size_t off) {
        PpcgRow<CPL> v;
        const size_t oc = off + s.c;
        v.x = ldrow<double, CPL>(X + oc);
        v.r = ldrow<double, CPL>(Rv + oc);
        v.u = ldrow<double, CPL>(U + oc);
        v.w = ldrow<double, CPL>(Wv + oc);
        // z, q, s, p are ignored on the first iteration (taken as zero)
        v.z = ldrow<double, CPL>(Z + oc);
        v.q = ldrow<double, CPL>(Q + oc);
        v.s = ldrow<double, CPL>(Sv + oc);
        v.p = ldrow<double, CPL>(Pp + oc);
        return v;
      },
      [&](size_t off, const R& hS, const R& hC, const R& hN, const R& W, const R& E,
          const R& B3, const R& T3, const auto& kc,
          const PpcgRow<CPL>& in) {
        R x = in.x, r = in.r, u = in.u, w = in.w, z, q, sv, p;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          const double nv = op_at<OP>(hS, hC, hN, W, E, B3, T3, kc, k);
          if (first) {
            z.e[k] = nv;
            q.e[k] = hC.e[k];
            sv.e[k] = w.e[k];
            p.e[k] = u.e[k];
          } else {
            z.e[k] = fma(be, in.z.e[k], nv);
            q.e[k] = fma(be, in.q.e[k], hC.e[k]);
            sv.e[k] = fma(be, in.s.e[k], w.e[k]);
            p.e[k] = fma(be, in.p.e[k], u.e[k]);
          }
          x.e[k] = fma(al, p.e[k], x.e[k]);
          r.e[k] = fma(nal, sv.e[k], r.e[k]);
          u.e[k] = fma(nal, q.e[k], u.e[k]);
          w.e[k] = fma(nal, z.e[k], w.e[k]);
          if (k < valid) {
            a0[k] = fma(r.e[k], u.e[k], a0[k]);
            a1[k] = fma(w.e[k], u.e[k], a1[k]);
            a2[k] = fma(r.e[k], r.e[k], a2[k]);
          }
        }
        const size_t oc = off + s.c;
        strow<double, CPL>(Z + oc, z, valid);
        strow<double, CPL>(Q + oc, q, valid);
        strow<double, CPL>(Sv + oc, sv, valid);
        strow<double, CPL>(Pp + oc, p, valid);
        strow<double, CPL>(X + oc, x, valid);
        strow<double, CPL>(Rv + oc, r, valid);
        strow<double, CPL>(U + oc, u, valid);
        strow<double, CPL>(Wv + oc, w, valid);
      });
  lv[0] = fold<CPL>(a0);
  lv[1] = fold<CPL>(a1);
  lv[2] = fold<CPL>(a2);
}

// --- K_CG1 / K_CG1F: p = r + beta p_old (on tile + halo); s = A p; store p;
//     slot (p, s).  First iteration: p = r.
template <typename T, int CPL, int OP = 0>
__device__ __forceinline__ void body_cg1(const PassArgs& a, int t, const Sc& sc, double* lv) {
  using R = Row<T, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  const T* Rv;
  const T* Po;
  T* Pn;
  if constexpr (sizeof(T) == 8) {
    Rv = a.r;
    Po = a.pc_in;
    Pn = a.pc_out;
  } else {
    Rv = a.rf;
    Po = a.pf_in;
    Pn = a.pf_out;
  }
  const T be = T(sc.be);
  const bool first = sc.first;
  double a0[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = 0.0;
  const int valid = g.nx - s.c;
  // the halo vector p = r + beta p_old is formed from the raw loads of r and
  // p_old when a row enters the window; on the first iteration p = r
  struct Raw {
    R r, po;
  };
  struct RawE {
    T r, po;
  };
  const EdgeAddr ea = edge_addr2<CPL>(s, g);
  auto hload = [=](size_t off) {
    Raw v;
    v.r = ldrow<T, CPL>(Rv + off + s.c);
    v.po = ldrow<T, CPL>(Po + off + s.c);  // ignored on the first iteration
    return v;
  };
  auto hmake = [=](const Raw& v) {
    R h;
#pragma unroll
    for (int k = 0; k < CPL; ++k) h.e[k] = first ? v.r.e[k] : fma(be, v.po.e[k], v.r.e[k]);
    return h;
  };
  auto walk_cg1 = [&](auto eload, auto emake, auto point, auto comp) {
    if constexpr (OP == 1) {
      auto hpart = [=](size_t off, int k) { return ldrow<T, CPL>((k ? Po : Rv) + off + s.c); };
      auto hjoin = [=](const R& r, const R& po) {
        Raw v;
        v.r = r;
        v.po = po;
        return hmake(v);
      };
      zwalk_split<T, CPL, CG1_PREFETCH>(g, s, hload, hmake, hpart, hjoin, eload, emake, point,
                                        comp);
    } else {
      walk<T, CPL, CG1_PREFETCH, OP, true>(g, s, hload, hmake, eload, emake, point, comp);
    }
  };
  walk_cg1(
      [=](size_t off) {
        RawE v;
#if EDGE_MASKED
        v.r = T(0);
        v.po = T(0);
        if (ea.emask) {
          v.r = Rv[off + ea.off];
          v.po = Po[off + ea.off];
        }
#else
        v.r = Rv[off + ea.off];
        v.po = Po[off + ea.off];
#endif
        return v;
      },
      [=](const RawE& v) { return ea.emask ? (first ? v.r : fma(be, v.po, v.r)) : T(0); },
      [](size_t) { return Empty{}; },
      [&](size_t off, const R& hS, const R& hC, const R& hN, const R& W, const R& E,
          const R& B3, const R& T3, const auto& kc,
          const Empty&) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          const T sv = op_at<OP>(hS, hC, hN, W, E, B3, T3, kc, k);
          if (k < valid) a0[k] = fma((double)hC.e[k], (double)sv, a0[k]);
        }
        strow<T, CPL>(Pn + off + s.c, hC, valid);
      });
  lv[0] = fold<CPL>(a0);
}

// --- K_CG2 / K_CG2X / K_CG2F: s = A p; x += alpha p; r -= alpha s; slot (r, r).
// XM: 0 = x (or d) untouched (odd iteration), 1 = x += alpha p (unused),
// 2 = x += alpha_prev p_prev, then x += alpha p (even iteration).  FP32: the
// inner solve's d, with alpha rounded to FP32 as in the oracle.
template <typename T, int CPL, int XM>
struct XrRow {
  Row<T, CPL> x, r, pp;
};

template <typename T, int CPL, int XM, int OP = 0>
__device__ __forceinline__ void body_cg2(const PassArgs& a, int t, const Sc& sc, double* lv) {
  using R = Row<T, CPL>;
  using In = XrRow<T, CPL, XM>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  const T* Pv;
  const T* Pp = nullptr;
  T* Xv;
  T* Rv;
  if constexpr (sizeof(T) == 8) {
    Pv = a.pc_in;
    Pp = a.pc_prev;
    Xv = a.x;
    Rv = a.r;
  } else {
    Pv = a.pf_in;
    Pp = a.pf_prev;
    Xv = a.df;
    Rv = a.rf;
  }
  const T al = T(sc.al), nal = -al, alp = T(sc.alp);
  double a0[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = 0.0;
  const int valid = g.nx - s.c;
  walk_plain<T, CPL, OP>(
      g, s, Pv,
      [=](size_t off) {
        In v;
        if constexpr (XM != 0) v.x = ldrow<T, CPL>(Xv + off + s.c);
        if constexpr (XM == 2) v.pp = ldrow<T, CPL>(Pp + off + s.c);
        v.r = ldrow<T, CPL>(Rv + off + s.c);
        return v;
      },
      [&](size_t off, const R& hS, const R& hC, const R& hN, const R& W, const R& E,
          const R& B3, const R& T3, const auto& kc,
          const In& in) {
        R x = in.x, r = in.r;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          const T sv = op_at<OP>(hS, hC, hN, W, E, B3, T3, kc, k);
          if constexpr (XM == 1) x.e[k] = fma(al, hC.e[k], x.e[k]);
          if constexpr (XM == 2) x.e[k] = fma(al, hC.e[k], fma(alp, in.pp.e[k], x.e[k]));
          r.e[k] = fma(nal, sv, r.e[k]);
          if (k < valid) a0[k] = fma((double)r.e[k], (double)r.e[k], a0[k]);
        }
        if constexpr (XM != 0) strow<T, CPL>(Xv + off + s.c, x, valid);
        strow<T, CPL>(Rv + off + s.c, r, valid);
      });
  lv[0] = fold<CPL>(a0);
}

// --- pending x update of a stopped solve: x += alp * P on tile t.
template <int CPL>
__device__ __forceinline__ void body_flush(const PassArgs& a, int t, const double* P,
                                           double alp) {
  using R = Row<double, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  const int valid = g.nx - s.c;
  if (valid <= 0) return;
  for (int j = s.j0; j < s.j1; j += s.js) {
    const size_t o = (size_t)j * g.pitch + s.c;
    const R pv = ldrow<double, CPL>(P + o);
    R x = ldrow<double, CPL>(a.x + o);
#pragma unroll
    for (int k = 0; k < CPL; ++k) x.e[k] = fma(alp, pv.e[k], x.e[k]);
    strow<double, CPL>(a.x + o, x, valid);
  }
}

// --- pending d update of a finished inner solve: d += alp * P (FP32).
__device__ __forceinline__ void body_flush_f32(const PassArgs& a, int t, const float* P,
                                               float alp) {
  using R = Row<float, 4>;
  const Geo& g = a.g;
  const Strip s = strip_of<4>(g, t);
  const int valid = g.nx - s.c;
  if (valid <= 0) return;
  for (int j = s.j0; j < s.j1; j += s.js) {
    const size_t o = (size_t)j * g.pitch + s.c;
    const R pv = ldrow<float, 4>(P + o);
    R d = ldrow<float, 4>(a.df + o);
#pragma unroll
    for (int k = 0; k < 4; ++k) d.e[k] = fmaf(alp, pv.e[k], d.e[k]);
    strow<float, 4>(a.df + o, d, valid);
  }
}

// The vector whose pending update a stopping pass of KIND applies: the
// pipelined p, pass 1's incoming direction, pass 2's previous direction.
template <int KIND>
__device__ __forceinline__ const double* flush_dir(const PassArgs& a) {
  if constexpr (KIND == K_PCG || KIND == K_PCGX) return a.p;
  else if constexpr (KIND == K_CG1 || KIND == K_CHEB) return a.pc_in;
  else return a.pc_prev;
}

template <int KIND>
__device__ __forceinline__ const float* flush_dir_f32(const PassArgs& a) {
  if constexpr (KIND == K_CG1F || KIND == K_CHEBF) return a.pf_in;
  else return a.pf_prev;
}

// Applies a stopped solve's pending update on tile t.
template <int KIND, int CPL>
__device__ __forceinline__ void run_flush(const PassArgs& a, int t, const Sc& sc) {
  if constexpr (inner_kind<KIND>()) body_flush_f32(a, t, flush_dir_f32<KIND>(a), float(sc.alp));
  else body_flush<CPL>(a, t, flush_dir<KIND>(a), sc.alp);
}

// --- K_REF_SCALE: rho = fp32((b - A x) * inv); d = 0; slot (rho, rho) in FP64.
template <int CPL, int OP = 0>
__device__ __forceinline__ void body_ref_scale(const PassArgs& a, int t, const Sc& sc,
                                               double* lv) {
  using R = Row<double, CPL>;
  using RF = Row<float, CPL>;
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  const double inv = sc.inv;
  double a0[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) a0[k] = 0.0;
  const int valid = g.nx - s.c;
  const double* B = a.b;
  float *Rf = a.rf, *Df = a.df;
  walk_plain<double, CPL, OP>(
      g, s, a.x, [=](size_t off) { return ldrow<double, CPL>(B + off + s.c); },
      [&](size_t off, const R& hS, const R& hC, const R& hN, const R& W, const R& E,
          const R& B3, const R& T3, const auto& kc,
          const R& bb) {
        RF rho;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          const double res = bb.e[k] - op_at<OP>(hS, hC, hN, W, E, B3, T3, kc, k);
          rho.e[k] = (float)(res * inv);
          if (k < valid) a0[k] = fma((double)rho.e[k], (double)rho.e[k], a0[k]);
        }
        strow<float, CPL>(Rf + off + s.c, rho, valid);
        strow<float, CPL>(Df + off + s.c, zrow<float, CPL>(), valid);
      });
  lv[0] = fold<CPL>(a0);
}

// --- K_REF_UPDATE: x += scale * fp64(d).
template <int CPL>
__device__ __forceinline__ void body_ref_update(const PassArgs& a, int t, const Sc& sc) {
  const Geo& g = a.g;
  const Strip s = strip_of<CPL>(g, t);
  const double sc_ = sc.al;
  const int valid = g.nx - s.c;
  for (int j = s.j0; j < s.j1; j += s.js) {
    const size_t o = (size_t)j * g.pitch + s.c;
    Row<double, CPL> x = ldrow<double, CPL>(a.x + o);
    const Row<float, CPL> d = ldrow<float, CPL>(a.df + o);
#pragma unroll
    for (int k = 0; k < CPL; ++k) x.e[k] = fma(sc_, (double)d.e[k], x.e[k]);
    strow<double, CPL>(a.x + o, x, valid);
  }
}

// OP != 0: the 7-point or the variable-coefficient operator (multi-work-group
// passes of the FP64 kinds only).
template <int KIND, int CPL, int OP = 0>
__device__ __forceinline__ void run_body(const PassArgs& a, int t, const Sc& sc, double* lv) {
  static_assert(OP == 0 || KIND == K_INIT_R || KIND == K_RESID || KIND == K_INIT_W ||
                    KIND == K_APPLY || KIND == K_DOT || KIND == K_PCG || KIND == K_PCGX ||
                    KIND == K_CG1 || KIND == K_CG2 || KIND == K_CG2X || KIND == K_RRQ ||
                    KIND == K_RRZ,
                "no form of this pass for the operator");
  if constexpr (OP != 0) {
    if constexpr (KIND == K_INIT_R) body_residual<CPL, true, OP>(a, t, lv);
    else if constexpr (KIND == K_RESID) body_residual<CPL, false, OP>(a, t, lv);
    else if constexpr (KIND == K_INIT_W) body_apply<CPL, true, OP>(a, t, lv);
    else if constexpr (KIND == K_APPLY || KIND == K_RRQ || KIND == K_RRZ)
      body_apply<CPL, false, OP>(a, t, lv);
    else if constexpr (KIND == K_DOT) body_dot<CPL>(a, t, lv);
    else if constexpr (KIND == K_PCG) body_pcg<CPL, false, OP>(a, t, sc, lv);
    else if constexpr (KIND == K_PCGX) body_pcg<CPL, true, OP>(a, t, sc, lv);
    else if constexpr (KIND == K_CG1) body_cg1<double, CPL, OP>(a, t, sc, lv);
    else if constexpr (KIND == K_CG2) body_cg2<double, CPL, 0, OP>(a, t, sc, lv);
    else if constexpr (KIND == K_CG2X) body_cg2<double, CPL, 2, OP>(a, t, sc, lv);
    return;
  }
  if constexpr (KIND == K_INIT_R) body_residual<CPL, true>(a, t, lv);
  else if constexpr (KIND == K_RESID) body_residual<CPL, false>(a, t, lv);
  else if constexpr (KIND == K_INIT_W) body_apply<CPL, true>(a, t, lv);
  else if constexpr (KIND == K_INIT_WU) body_init_wu<CPL>(a, t, lv);
  else if constexpr (KIND == K_PPCG) body_ppcg<CPL>(a, t, sc, lv);
  else if constexpr (KIND == K_APPLY || KIND == K_RRQ || KIND == K_RRZ)
    body_apply<CPL, false>(a, t, lv);
  else if constexpr (KIND == K_DOT) body_dot<CPL>(a, t, lv);
  else if constexpr (KIND == K_PCG) body_pcg<CPL, false>(a, t, sc, lv);
  else if constexpr (KIND == K_PCGX) body_pcg<CPL, true>(a, t, sc, lv);
  else if constexpr (KIND == K_CG1) body_cg1<double, CPL>(a, t, sc, lv);
  else if constexpr (KIND == K_CG2) body_cg2<double, CPL, 0>(a, t, sc, lv);
  else if constexpr (KIND == K_CG2X) body_cg2<double, CPL, 2>(a, t, sc, lv);
  else if constexpr (KIND == K_CG1F) body_cg1<float, CPL>(a, t, sc, lv);
  else if constexpr (KIND == K_CG2F) body_cg2<float, CPL, 0>(a, t, sc, lv);
  else if constexpr (KIND == K_CG2FX) body_cg2<float, CPL, 2>(a, t, sc, lv);
  else if constexpr (KIND == K_REF_SCALE) body_ref_scale<CPL>(a, t, sc, lv);
  else if constexpr (KIND == K_REF_UPDATE) body_ref_update<CPL>(a, t, sc);
}

// The body of KIND with the x variant the transition chose (for paths that
// decide on the device: the single-work-group solver and the step kernel).
template <int KIND, int CPL, int OP = 0>
__device__ __forceinline__ void run_body_any(const PassArgs& a, int t, const Sc& sc, double* lv) {
  if constexpr (KIND == K_PCG) {
    if (sc.xu) run_body<K_PCGX, CPL, OP>(a, t, sc, lv);
    else run_body<K_PCG, CPL, OP>(a, t, sc, lv);
  } else if constexpr (KIND == K_CG2) {
    if (sc.xu) run_body<K_CG2X, CPL, OP>(a, t, sc, lv);
    else run_body<K_CG2, CPL, OP>(a, t, sc, lv);
  } else if constexpr (KIND == K_CG2F) {
    if (sc.xu) run_body<K_CG2FX, CPL, OP>(a, t, sc, lv);
    else run_body<K_CG2F, CPL, OP>(a, t, sc, lv);
  } else {
    run_body<KIND, CPL, OP>(a, t, sc, lv);
  }
}

// LDS per tile group: 4*2 doubles for the cross-tile stage, then 2*4*D for
// the tiles of a pass with D <= 3 slots (at offset 8).
constexpr int kLdsPerGroup = 4 * 2 + 2 * 4 * 3;

// ------------------------------------------------------ multi-group pass --
//
// grid = G work-groups of 256 threads, G a multiple of 8.  Work-group b is
// placed by the hardware on XCD b % 8; the tiles are split into 8 contiguous
// bands, band x served by the work-groups of XCD x, so vertically adjacent
// tiles (whose halo rows overlap) share an L2.  Every other pass walks each
// band in reverse order, so a pass starts on the tiles the previous pass
// wrote last, while they are still in the memory-side cache.  The order in
// which tiles are processed does not change any result: partials are stored
// per tile and summed in tile order.
template <int KIND, int CPL, int OP = 0>
__global__ __launch_bounds__(kGroup) void k_pass(PassArgs a) {
  __shared__ double lds[kLdsPerGroup];
  constexpr int DI = ndots_in<KIND>(), DO = ndots_out<KIND>();
  Sc sc;
  if constexpr (KIND == K_APPLY || KIND == K_DOT) {
    sc.al = sc.be = sc.inv = sc.alp = 0.0;
    sc.first = 0;
    sc.xu = 0;
  } else {
    State s = load_state_uniform(a.st_in);
    double sum[2] = {0.0, 0.0};
    if constexpr (DI > 0) {
      // classic pass 1 takes (b,b) too after the initial residual; with the
      // preconditioner its one slot is (r,z) in the Chebyshev pass's tiles
      const bool pc = (KIND == K_CG1 || KIND == K_CG1F) && (s.flags & F_PRECOND);
      const int din = (KIND == K_CG1) ? ((s.flags & F_BB_PENDING) && !pc ? 2 : 1) : DI;
      const int tin = pc ? a.cheb_tiles : a.g.tiles;
      if (s.status == ST_RUNNING) {
        if (din == 2) cross_tile_sum<2>(a.part_in, tin, sum, lds);
        else cross_tile_sum<1>(a.part_in, tin, sum, lds);
      }
      sum[0] = uniform(sum[0]);
      sum[1] = uniform(sum[1]);
    }
    bool flush = false;
    const bool run = transition_x<KIND>(s, sum, sc, flush);
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.st_out = s;
    if constexpr (defers_x<KIND>()) {
      if (flush) {
        // this pass stopped the solve after an odd iteration: apply its update
        const int G = gridDim.x, b = blockIdx.x;
        const int xcd = b & 7, slot = b >> 3, nb = G >> 3;
        const int T = a.g.tiles;
        const int t0 = (int)(((int64_t)T * xcd) >> 3), t1 = (int)(((int64_t)T * (xcd + 1)) >> 3);
        for (int t = t0 + slot; t < t1; t += nb) run_flush<KIND, CPL>(a, t, sc);
        return;
      }
    }
    if (!run) return;
  }

  const int G = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3, nb = G >> 3;
  const int T = a.g.tiles;
  const int t0 = (int)(((int64_t)T * xcd) >> 3), t1 = (int)(((int64_t)T * (xcd + 1)) >> 3);
  int par = 0;
  for (int tt = t0 + slot; tt < t1; tt += nb, par ^= 1) {
    const int t = a.rev ? t1 - 1 - (tt - t0) : tt;
    double lv[DO > 2 ? DO : 2];
    run_body<KIND, CPL, OP>(a, t, sc, lv);
    if constexpr (DO > 0) tile_partial<DO>(lv, a.part_out, T, t, lds + 8, par);
  }
}

// res2 = cross-tile sum of slot 0 (true residual at exit); one work-group.
__global__ __launch_bounds__(kGroup) void k_final(PassArgs a) {
  __shared__ double lds[8];
  double sum[1];
  cross_tile_sum<1>(a.part_in, a.g.tiles, sum, lds);
  if (threadIdx.x == 0) {
    State s = *a.st_in;
    s.res2 = sum[0];
    *a.st_out = s;
  }
}

// ---------------------------------------------- Chebyshev preconditioner --
//
// z = p_s(A) r: s steps of Chebyshev semi-iteration on A y = r from y = 0
// (d_0 = c0 r, y_1 = d_0; r_k = r_(k-1) - A d_(k-1), d_k = fma(c1_k, d_(k-1),
// c2_k r_k), y_(k+1) = y_k + d_k), the coefficients from the spectrum
// interval of the operator (computed on the host).  The stencil, the fma
// structure and the order of the y sums are those of the oracle's canonical
// mode, so z is bitwise the oracle's whatever the blocking.
//
// Temporal blocking in registers.  A wavefront owns 128 consecutive columns
// (lane l: columns cl = cw - 8 + 2l and cl + 1) and marches down the rows of
// its item.  Stage k of step J computes row J - k of r_k, d_k and adds d_k
// into y: stage 0 scales the row just loaded, stage k >= 1 applies the
// stencil to d_(k-1) on rows J-k-1 .. J-k+1, the last of which stage k - 1
// produced in the same step.  Each level keeps only its two newest rows of
// d and its newest row of r, y keeps the s - 1 rows still accumulating, and
// row J - (s - 1) of z is complete after step J.  West and east neighbours
// come from the adjacent lanes (DPP); values near the wavefront's outer
// columns lose one valid column per stage, so of the 128 columns the middle
// 112 (the 8-column halo >= s - 1 on each side) are written.  Cells outside
// the grid are held at zero through every stage (`MASK`, only for the
// wavefronts and items that touch the grid edge).
//
// Items and partials.  A work-group of 8 wavefronts covers 8 x 112 = 896
// columns, exactly 7 tiles of 128 columns, over the rows [ty H, (ty+1) H) of
// one item (H = cheb_rows).  (r, z) is reduced in the tile order of a tile
// 128 columns wide and H rows tall holding one wavefront: each lane
// accumulates its two columns with fma down the rows, the wavefronts park
// the column sums in LDS, and wavefront m folds the column pair of each lane
// of tile m, butterflies, and stores partial[ty ntx + tx].
constexpr int kChebHaloCols = 8;                                       // >= s - 1
constexpr int kChebOut = 2 * kWave - 2 * kChebHaloCols;                // 112
constexpr int kChebWaves = 8;
constexpr int kChebThreads = kChebWaves * kWave;
constexpr int kChebGroupTiles = kChebWaves * kChebOut / (2 * kWave);   // 7
static_assert(kChebGroupTiles * 2 * kWave == kChebWaves * kChebOut, "whole tiles per group");
static_assert(kChebHaloCols >= kChebMaxSteps - 1, "halo too narrow for the steps");
static_assert(kChebGroupCols == kChebWaves * kChebOut, "item width known to the host");

// A lane's two columns, binary64 (the FP64 solves) or binary32 (the inner
// solve of the refinement), and the matching vector load type.
template <typename T>
struct V2 {
  T v[2];
};
template <typename T>
using Pair = std::conditional_t<sizeof(T) == 8, double2, float2>;

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int clcm(int a, int b) { return a / cgcd(a, b) * b; }
constexpr int cmod(int a, int m) { return ((a % m) + m) % m; }

// Lane shifts with zero fill (bound_ctrl): lane l receives lane l-1 (shr) or
// lane l+1 (shl); lane 0 (shr) and lane 63 (shl) receive 0.
template <int CTRL>
__device__ __forceinline__ double dpp0(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp0(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

// One wavefront of an item: output columns [cw, cw + 112), rows [y0, y1).
// Rows are numbered from Jb = y0 - (s - 1); every ring below is indexed by
// the row modulo its length, and the row loop is expanded over a period that
// all the lengths divide (one step per template instance), so the rings
// never move in registers.
template <int S, typename T>
struct ChebRegs {
  static constexpr int H = S - 1;            // stencil steps = halo rows
  static constexpr int L = H > 0 ? H : 1;    // y / r ring length
  static constexpr int PD = S <= 3 ? 4 : 2;  // rows loaded ahead
  static constexpr int P = clcm(clcm(2, L), PD);
  // (r, z) needs r on row J-H at step J: kept in registers up to s = 6, read
  // again (a cache hit: this wavefront read that row H steps before) one
  // step ahead beyond, where the registers are needed for the stages
  static constexpr bool RELOAD = S >= 7;
  static constexpr int LR = RELOAD ? 1 : L;
  V2<T> d[L][2];    // d_k on rows J-k-2, J-k-1 (slot (row - Jb) mod 2), levels k < H
  V2<T> rk[L][2];   // r_k on row J-k-1 (same slots)
  V2<T> y[L];       // y on rows J-H .. J-1 (slot (row - Jb) mod L)
  V2<T> r0[LR];     // r on the same rows, for (r, z) (RELOAD: unused)
  V2<T> rr[2];      // RELOAD: r on rows J-H, J-H+1 (slot (row - Jb) mod 2)
  V2<T> ld[PD];     // r loaded for rows J .. J+PD-1 (slot (row - Jb) mod PD)
  double a0, a1; // (r, z) column sums
};

template <typename T>
struct ChebCtx {
  const T* R;  // r + first column of the lane
  T* Z;        // z + first column of the lane
  int pitch, ny, y0, Je;
  bool v0, v1, outl;
};

template <bool MASK, typename T>
__device__ __forceinline__ V2<T> cheb_load(const ChebCtx<T>& c, int J) {
  const int jl = min(max(J, 0), c.ny - 1);
  const Pair<T> t = *reinterpret_cast<const Pair<T>*>(c.R + (size_t)jl * c.pitch);
  V2<T> o;
  o.v[0] = t.x;
  o.v[1] = t.y;
  if constexpr (MASK) {
    const bool rv = J >= 0 && J < c.ny;
    o.v[0] = (rv && c.v0) ? o.v[0] : T(0);
    o.v[1] = (rv && c.v1) ? o.v[1] : T(0);
  }
  return o;
}

// Step J = J0 + Q of the march; false once the item's rows are exhausted.
template <int S, bool MASK, int Q, typename T>
__device__ __forceinline__ bool cheb_step(const ChebCtx<T>& c, const T* c1, const T* c2, T c0,
                                          ChebRegs<S, T>& g, int J0) {
  using G = ChebRegs<S, T>;
  constexpr int H = G::H, L = G::L, PD = G::PD;
  const int J = J0 + Q;
  if (J >= c.Je) return false;
  const V2<T> rin = g.ld[Q % PD];
  g.ld[Q % PD] = cheb_load<MASK>(c, J + PD);
  V2<T> rrow;
  if constexpr (G::RELOAD) {
    rrow = g.rr[cmod(Q - H, 2)];
    g.rr[cmod(Q - H + 1, 2)] = cheb_load<MASK>(c, J - H + 1);
  }
  // stage 0: d_0 = c0 r, y = d_0 on row J (zero outside the grid already)
  V2<T> dn, rn = rin, ynew;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    dn.v[e] = rin.v[e] * c0;
    ynew.v[e] = dn.v[e];
  }
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    // stage k on row J - k from level k-1: rows J-k-1 (slot so), J-k
    // (slot sc) and J-k+1 (dn, this step)
    const int so = cmod(Q - (k - 1), 2), sc = so ^ 1;
    const V2<T> C = g.d[k - 1][sc], Sv = g.d[k - 1][so], Nv = dn;
    const T w0 = dpp0<kDppWaveShr1>(C.v[1]);
    const T e1 = dpp0<kDppWaveShl1>(C.v[0]);
    const T W[2] = {w0, C.v[0]}, E[2] = {C.v[1], e1};
    V2<T> dk, rk;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const T t = st5(C.v[e], W[e], E[e], Sv.v[e], Nv.v[e]);
      rk.v[e] = g.rk[k - 1][sc].v[e] - t;
      dk.v[e] = fma(c1[k - 1], C.v[e], c2[k - 1] * rk.v[e]);
    }
    if constexpr (MASK) {
      const int j = J - k;
      const bool rv = j >= 0 && j < c.ny;
      dk.v[0] = (rv && c.v0) ? dk.v[0] : T(0);
      dk.v[1] = (rv && c.v1) ? dk.v[1] : T(0);
    }
    V2<T>& yk = g.y[cmod(Q - k, L)];
#pragma unroll
    for (int e = 0; e < 2; ++e) yk.v[e] = yk.v[e] + dk.v[e];
    // level k-1's row J-k+1 replaces its row J-k-1 (used just now)
    g.d[k - 1][so] = dn;
    g.rk[k - 1][so] = rn;
    dn = dk;
    rn = rk;
  }
  // row J - H of z is complete (slot Q mod L, which row J takes next)
  constexpr int os = Q % L;
  const V2<T> zrow = H > 0 ? g.y[os] : ynew;
  if constexpr (!G::RELOAD) rrow = H > 0 ? g.r0[os] : rin;
  if (J >= c.y0 + H) {
    if (c.outl) {
      Pair<T> o;
      o.x = zrow.v[0];
      o.y = zrow.v[1];
      *reinterpret_cast<Pair<T>*>(c.Z + (size_t)(J - H) * c.pitch) = o;
    }
    // (r, z) in binary64 for both element types
    g.a0 = fma((double)rrow.v[0], (double)zrow.v[0], g.a0);
    g.a1 = fma((double)rrow.v[1], (double)zrow.v[1], g.a1);
  }
  if constexpr (H > 0) {
    g.y[os] = ynew;
    if constexpr (!G::RELOAD) g.r0[os] = rin;
  }
  return true;
}

template <int S, bool MASK, typename T, int... Qs>
__device__ __forceinline__ bool cheb_period(const ChebCtx<T>& c, const T* c1, const T* c2, T c0,
                                            ChebRegs<S, T>& g, int J0,
                                            std::integer_sequence<int, Qs...>) {
  return (cheb_step<S, MASK, Qs>(c, c1, c2, c0, g, J0) && ...);
}

// R is the input vector, Z the output; ntx the 128-column tiles across the
// padded row.  acc0/acc1 receive the (r, z) column sums of the lane's two
// columns.
template <int S, bool MASK, typename T>
__device__ __forceinline__ void cheb_march(const PassArgs& a, const T* R, T* Z, int ntx, int cw,
                                           int y0, int y1, double& acc0, double& acc1) {
  using G = ChebRegs<S, T>;
  constexpr int H = G::H, L = G::L, PD = G::PD, P = G::P;
  const Geo& gg = a.g;
  const int lane = threadIdx.x & (kWave - 1);
  const int cl = cw - kChebHaloCols + 2 * lane;
  // the coefficients are uniform: scalar registers (binary32: each rounded
  // once from the binary64 coefficient)
  const T c0 = T(uniform(a.cheb[0]));
  T c1[L], c2[L];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    c1[k] = T(uniform(a.cheb[1 + k]));
    c2[k] = T(uniform(a.cheb[S + k]));
  }
  ChebCtx<T> c;
  // columns: the load address is valid for 0 <= cl < the padded row length
  // (a multiple of 128; cl is even, so the pair stays in the row)
  c.v0 = c.v1 = true;
  int lc = cl;
  if constexpr (MASK) {
    c.v0 = cl >= 0 && cl < gg.nx;
    c.v1 = cl >= 0 && cl + 1 < gg.nx;
    lc = (cl >= 0 && cl < ntx * 2 * kWave) ? cl : 0;
  }
  c.R = R + lc;
  c.Z = Z + cl;
  c.pitch = gg.pitch;
  c.ny = gg.ny;
  c.y0 = y0;
  c.Je = y1 + H;
  c.outl = lane >= kChebHaloCols / 2 && lane < kWave - kChebHaloCols / 2 && (!MASK || cl < gg.nx);
  G g;
#pragma unroll
  for (int k = 0; k < L; ++k)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      g.d[k][0].v[e] = g.d[k][1].v[e] = g.rk[k][0].v[e] = g.rk[k][1].v[e] = T(0);
      g.y[k].v[e] = T(0);
    }
#pragma unroll
  for (int k = 0; k < G::LR; ++k) g.r0[k].v[0] = g.r0[k].v[1] = T(0);
  g.rr[0] = g.rr[1] = g.r0[0];
  g.a0 = g.a1 = 0.0;
  const int Jb = y0 - H;
#pragma unroll
  for (int i = 0; i < PD; ++i) g.ld[i] = cheb_load<MASK>(c, Jb + i);
  for (int J0 = Jb; J0 < c.Je; J0 += P)
    if (!cheb_period<S, MASK>(c, c1, c2, c0, g, J0, std::make_integer_sequence<int, P>{})) break;
  acc0 = g.a0;
  acc1 = g.a1;
}

// Chebyshev tiles (128 columns) across the padded row: the FP64 tile passes'
// tiles are 128 columns wide, the FP32 ones (4 columns per lane) 256.
template <typename T>
__device__ __forceinline__ int cheb_ntx(const Geo& g) {
  return sizeof(T) == 8 ? g.ntx : 2 * g.ntx;
}

// Chebyshev item `it` (ngx items across): each wavefront marches its 112
// output columns over the item's rows; without PIPE the (r, z) column sums
// become one partial per 128-column tile (wavefront m folds tile m).
// `colacc` holds kChebWaves * kChebOut doubles.  FP64: a.r -> a.z; FP32 (the
// refinement's inner solve): a.rf -> a.zf.
template <int S, bool PIPE, typename T = double>
__device__ __forceinline__ void cheb_item(const PassArgs& a, int it, int ngx, double* colacc) {
  const Geo& g = a.g;
  const int ntx = cheb_ntx<T>(g);
  const T* R;
  T* Z;
  if constexpr (sizeof(T) == 8) {
    R = a.r;
    Z = a.z;
  } else {
    R = a.rf;
    Z = a.zf;
  }
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
  const int Hc = a.cheb_rows;
  const int gx = it % ngx, ty = it / ngx;
  const int cw = gx * (kChebGroupTiles * 2 * kWave) + wave * kChebOut;
  const int y0 = ty * Hc, y1 = min(y0 + Hc, g.ny);
  double acc0 = 0.0, acc1 = 0.0;
  if (cw < g.nx) {
    const bool inner = cw >= kChebHaloCols && cw + kChebOut + kChebHaloCols <= g.nx &&
                       y0 >= S - 1 && y1 + (S - 1) <= g.ny;
    if (inner) cheb_march<S, false>(a, R, Z, ntx, cw, y0, y1, acc0, acc1);
    else cheb_march<S, true>(a, R, Z, ntx, cw, y0, y1, acc0, acc1);
  }
  // PIPE: no partials, the fused pass sums its dots.  The column sums are
  // still formed: without them the compiler schedules the march of s = 8
  // into more than 256 registers and spills.
  if constexpr (PIPE) __asm__ volatile("" ::"v"(acc0), "v"(acc1));
  if (!PIPE && lane >= kChebHaloCols / 2 && lane < kWave - kChebHaloCols / 2) {
    double* c = colacc + wave * kChebOut + 2 * (lane - kChebHaloCols / 2);
    c[0] = acc0;
    c[1] = acc1;
  }
  __syncthreads();
  if (!PIPE && wave < kChebGroupTiles) {
    const int tx = gx * kChebGroupTiles + wave;
    if (tx < ntx) {
      const double* c = colacc + wave * 2 * kWave + 2 * lane;
      const double v = wave_sum(c[0] + c[1]);
      if (lane == 0) a.part_out[(size_t)ty * ntx + tx] = v;
    }
  }
  __syncthreads();
}

// PIPE = false: K_CHEB (z = M^-1 r of classic CG, and of the pipelined
// variant's first residual); PIPE = true: K_CHEBW (m = M^-1 w of the
// pipelined variant, after its scalar step; no partials).  The input vector
// is a.r, the output a.z.
template <int S, bool PIPE>
__global__ __launch_bounds__(kChebThreads) void k_cheb(PassArgs a) {
  __shared__ double colacc[kChebWaves * kChebOut];
  __shared__ double red[4 * 3];
  {
    State s = load_state_uniform(a.st_in);
    double sum[3] = {0.0, 0.0, 0.0};
    if (s.status == ST_RUNNING) {
      if (PIPE) cross_tile_sum<3>(a.part_in, a.g.tiles, sum, red);
      else if (s.flags & F_BB_PENDING) cross_tile_sum<2>(a.part_in, a.g.tiles, sum, red);
      else cross_tile_sum<1>(a.part_in, a.g.tiles, sum, red);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) sum[d] = uniform(sum[d]);
    Sc sc;
    bool flush = false;
    const bool run = PIPE ? transition<K_CHEBW>(s, sum, sc)
                          : transition_x<K_CHEB>(s, sum, sc, flush);
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.st_out = s;
    if (flush) {
      // the stop test stopped the solve after an odd iteration: apply that
      // iteration's x update (pass tiles, 256 threads per tile)
      if (threadIdx.x < kGroup) {
        const int G = gridDim.x, b = blockIdx.x;
        const int xcd = b & 7, slot = b >> 3, nb = G >> 3;
        const int T = a.g.tiles;
        const int t0 = (int)(((int64_t)T * xcd) >> 3), t1 = (int)(((int64_t)T * (xcd + 1)) >> 3);
        for (int t = t0 + slot; t < t1; t += nb) run_flush<K_CHEB, 2>(a, t, sc);
      }
      return;
    }
    if (!run) return;
  }
  const Geo& g = a.g;
  const int ngx = (g.ntx + kChebGroupTiles - 1) / kChebGroupTiles;
  const int Hc = a.cheb_rows, nty = (g.ny + Hc - 1) / Hc;
  const int I = ngx * nty;
  const int G = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3, nb = G >> 3;
  const int i0 = (int)(((int64_t)I * xcd) >> 3), i1 = (int)(((int64_t)I * (xcd + 1)) >> 3);
  for (int it = i0 + slot; it < i1; it += nb) cheb_item<S, PIPE>(a, it, ngx, colacc);
}

// K_CHEBF: z = M^-1 r of the refinement's preconditioned inner solve, in
// binary32 (a.rf -> a.zf, (r, z) partials per 128-column tile as in K_CHEB).
// The prologue makes the inner stop test on (r, r) of the inner residual
// (the scale pass or pass 2 before it) and, when that test ends the inner
// solve after an odd inner iteration, applies its pending d update instead.
template <int S>
__global__ __launch_bounds__(kChebThreads) void k_chebf(PassArgs a) {
  __shared__ double colacc[kChebWaves * kChebOut];
  __shared__ double red[4];
  {
    State s = load_state_uniform(a.st_in);
    double sum[1] = {0.0};
    if (s.status == ST_RUNNING) cross_tile_sum<1>(a.part_in, a.g.tiles, sum, red);
    sum[0] = uniform(sum[0]);
    Sc sc;
    bool flush = false;
    const bool run = transition_x<K_CHEBF>(s, sum, sc, flush);
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.st_out = s;
    if (flush) {
      if (threadIdx.x < kGroup) {
        const int G = gridDim.x, b = blockIdx.x;
        const int xcd = b & 7, slot = b >> 3, nb = G >> 3;
        const int T = a.g.tiles;
        const int t0 = (int)(((int64_t)T * xcd) >> 3), t1 = (int)(((int64_t)T * (xcd + 1)) >> 3);
        for (int t = t0 + slot; t < t1; t += nb) run_flush<K_CHEBF, 4>(a, t, sc);
      }
      return;
    }
    if (!run) return;
  }
  const Geo& g = a.g;
  const int ngx = (cheb_ntx<float>(g) + kChebGroupTiles - 1) / kChebGroupTiles;
  const int Hc = a.cheb_rows, nty = (g.ny + Hc - 1) / Hc;
  const int I = ngx * nty;
  const int G = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3, nb = G >> 3;
  const int i0 = (int)(((int64_t)I * xcd) >> 3), i1 = (int)(((int64_t)I * (xcd + 1)) >> 3);
  for (int it = i0 + slot; it < i1; it += nb) cheb_item<S, false, float>(a, it, ngx, colacc);
}

__global__ void k_fill(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ------------------------------------------------- single work-group solve --
//
// The whole solve inside one work-group of kWgGroups tile groups for small
// grids: the same pass bodies and the same reduction order as the
// multi-work-group path, separated by work-group barriers instead of kernel
// boundaries.  Group g handles tiles g, g+kWgGroups, ...; every group
// evaluates the cross-tile stage itself (identical result).  Buffers: part_in/part_out are
// the two partial buffers, w_in/w_out (pipelined) or pc_in/pc_out (classic)
// the two halo buffers; st_in is the initial state, st_out the final one.
template <int KIND>
__device__ __forceinline__ void wg_pass(const PassArgs& a, const Sc& sc, double* lds) {
  constexpr int DO = ndots_out<KIND>();
  static_assert(DO <= 2, "passes with three slots run only as multi-work-group passes");
  const int grp = threadIdx.x >> 8;
  const int T = a.g.tiles;
  // every group runs the same number of tile iterations (barrier balance)
  const int iters = (T + kWgGroups - 1) / kWgGroups;
  for (int i = 0, par = 0; i < iters; ++i, par ^= 1) {
    const int t = grp + kWgGroups * i;
    double lv[2] = {0.0, 0.0};
    if (t < T) run_body_any<KIND, 2>(a, t, sc, lv);
    if constexpr (DO > 0) {
      // groups past the end join the barrier but store nothing
      const int tid = threadIdx.x & (kGroup - 1), lane = tid & 63, wave = tid >> 6;
      double* L = lds + par * kWavesPerTile * DO;
#pragma unroll
      for (int d = 0; d < DO; ++d) {
        const double v = wave_sum(lv[d]);
        if (lane == 0) L[wave * DO + d] = v;
      }
      __syncthreads();
      if (tid == 0 && t < T) {
#pragma unroll
        for (int d = 0; d < DO; ++d) {
          double s = L[d];
#pragma unroll
          for (int w = 1; w < kWavesPerTile; ++w) s = s + L[w * DO + d];
          a.part_out[(size_t)d * T + t] = s;
        }
      }
    }
  }
  __syncthreads();  // vectors and partials of this pass visible to the next
}

template <int KIND>
__device__ __forceinline__ bool wg_step(State& s, const PassArgs& a, Sc& sc, double* lds) {
  constexpr int DI = ndots_in<KIND>();
  double sum[2] = {0.0, 0.0};
  if (DI > 0 && s.status == ST_RUNNING) {
    const int din = (KIND == K_CG1) ? ((s.flags & F_BB_PENDING) ? 2 : 1) : DI;
    if (din == 2) cross_tile_sum<2>(a.part_in, a.g.tiles, sum, lds);
    else cross_tile_sum<1>(a.part_in, a.g.tiles, sum, lds);
  }
  bool flush = false;
  const bool run = transition_x<KIND>(s, sum, sc, flush);
  if constexpr (defers_x<KIND>()) {
    if (flush) {
      const int grp = threadIdx.x >> 8;
      for (int t = grp; t < a.g.tiles; t += kWgGroups) run_flush<KIND, 2>(a, t, sc);
      __syncthreads();  // x complete before the final residual reads it
    }
  }
  if (run) wg_pass<KIND>(a, sc, lds + 8);
  return run;
}

constexpr int kWgMaxLdsTiles = 64;  // up to this many tiles the partials stay in LDS

template <int VARIANT>
__global__ __launch_bounds__(kWgGroups * kGroup) void k_solve_wg(PassArgs a0) {
  __shared__ double lds_all[kWgGroups * kLdsPerGroup];
  __shared__ double lds_part[2][2 * kWgMaxLdsTiles];
  double* lds = lds_all + (threadIdx.x >> 8) * kLdsPerGroup;
  State s = *a0.st_in;
  // the per-tile partials of a pass live in LDS for small grids (the same
  // values and order as in global memory, one L2 round trip less per pass)
  const bool in_lds = a0.g.tiles <= kWgMaxLdsTiles;
  double* P0 = in_lds ? lds_part[0] : const_cast<double*>(a0.part_in);
  double* P1 = in_lds ? lds_part[1] : a0.part_out;
  Sc sc;
  PassArgs a = a0;
  // r = b - A x
  a.part_out = P0;
  wg_step<K_INIT_R>(s, a, sc, lds);
  double* cur = P0;  // partials produced by the last pass
  double* nxt = P1;
  if constexpr (VARIANT == 1) {
    a.part_in = cur;
    a.part_out = nxt;
    a.w_out = const_cast<double*>(a0.w_in);
    if (wg_step<K_INIT_W>(s, a, sc, lds)) {
      double* t = cur; cur = nxt; nxt = t;
    }
    const double* Wi = a0.w_in;
    double* Wo = a0.w_out;
    while (s.status == ST_RUNNING) {
      a.part_in = cur;
      a.part_out = nxt;
      a.w_in = Wi;
      a.w_out = Wo;
      if (!wg_step<K_PCG>(s, a, sc, lds)) break;
      double* t = cur; cur = nxt; nxt = t;
      const double* tw = Wi; Wi = Wo; Wo = const_cast<double*>(tw);
    }
  } else {
    const double* Pi = a0.pc_in;
    double* Po = a0.pc_out;
    while (s.status == ST_RUNNING) {
      a.part_in = cur;
      a.part_out = nxt;
      a.pc_in = Pi;
      a.pc_out = Po;
      if (!wg_step<K_CG1>(s, a, sc, lds)) break;
      { double* t = cur; cur = nxt; nxt = t; }
      a.part_in = cur;
      a.part_out = nxt;
      a.pc_in = Po;
      a.pc_prev = Pi;
      if (!wg_step<K_CG2>(s, a, sc, lds)) break;
      { double* t = cur; cur = nxt; nxt = t; }
      const double* tp = Pi; Pi = Po; Po = const_cast<double*>(tp);
    }
  }
  // true residual of the final iterate
  if (s.status != ST_ZERO_RHS) {
    a.part_out = nxt;
    wg_step<K_RESID>(s, a, sc, lds);
    double sum[1];
    cross_tile_sum<1>(nxt, a.g.tiles, sum, lds);
    s.res2 = sum[0];
  }
  if (threadIdx.x == 0) *a0.st_out = s;
}

// ------------------------------------------ register-resident small solve --
//
// For a grid with (nx + 1) * ceil(ny / kRrRows) <= kRrThreads the whole solve
// runs in one work-group with every vector on chip.  Threads are laid out in
// rows of nx + 1: thread t owns column c = t mod (nx + 1) and the kRrRows rows
// of segment t div (nx + 1) (rows past ny are held as zero); the last thread
// of each row (c == nx) and the threads past the last segment own nothing and
// hold zeros, so the west neighbour of column 0 and the east neighbour of
// column nx-1 read as zero without a test.  Along a column the stencil's
// south/north neighbours are the thread's own registers; west/east neighbours
// come from the adjacent lanes by DPP.  What crosses a thread's boundary (the
// first and last element of every segment, the whole segment of lanes 0 and
// 63 of each wavefront) goes through LDS, together with the wavefront sums of
// the dot products, with one barrier per exchange and the LDS buffers
// double-buffered by phase parity.  Pipelined CG keeps x in LDS (six vectors
// do not fit the register file), classic CG keeps all four of its vectors
// (x, r, p, A p) in registers.
//
// Rows outside the grid hold exact zeros through every update (the stencil
// result is forced to zero there, and every other update maps zeros to +0),
// so the dot products accumulate them without a test: fma(0, 0, acc) == acc.
//
// Dot products follow the column-segment order: fma per thread over its rows
// in ascending order, xor butterfly, wavefronts in order.  The scalar
// recurrences are the transitions of the pass kernels, and every vector
// update is the same expression as in the pass bodies.

constexpr int kRrWaves = kRrThreads / kWave;

struct RrXchg {  // one exchanged vector
  double first[kRrThreads];  // element 0 of each thread's segment
  double last[kRrThreads];   // element kRrRows-1
  // segments of lanes 0 and 63 of wavefront w at [w + 1]; [0] stays zero (the
  // west neighbour of thread 0)
  double edge[kRrWaves + 1][2][kRrRows];
};

struct RrLdsPcg {
  RrXchg x[2];                     // by phase parity
  double tot[2][kRrWaves][2];      // wavefront sums, by phase parity
  double xs[kRrRows][kRrThreads];  // the iterate x
};

struct RrLdsCg {
  RrXchg x[2][2];  // [parity][r, p]
  double tot[2][kRrWaves][2];
};

constexpr size_t kRrLdsBytes =
    sizeof(RrLdsPcg) > sizeof(RrLdsCg) ? sizeof(RrLdsPcg) : sizeof(RrLdsCg);

struct RrSeg {
  int t, lane, wave, nw;
  int stride;         // threads per row of segments (nx + 1)
  int nv;             // rows of the segment inside the grid (0: idle thread)
  bool south, north;  // the segment below / above exists
  size_t off;         // element offset of the segment's first row (padded pitch)
  int pitch;
};

__device__ __forceinline__ RrSeg rr_seg(const Geo& g) {
  RrSeg s;
  s.t = threadIdx.x;
  s.lane = s.t & (kWave - 1);
  s.wave = s.t >> 6;
  s.nw = blockDim.x >> 6;
  s.stride = g.nx + 1;
  const int nseg = (g.ny + kRrRows - 1) / kRrRows;
  const int c = s.t % s.stride, sg = s.t / s.stride;
  const bool act = sg < nseg && c < g.nx;
  s.nv = act ? min(kRrRows, g.ny - sg * kRrRows) : 0;
  s.south = act && sg > 0;
  s.north = act && sg + 1 < nseg;
  s.pitch = g.pitch;
  s.off = act ? (size_t)sg * kRrRows * g.pitch + c : 0;
  return s;
}

// Zeroes the never-written edge entry of both parities of an exchange buffer.
__device__ __forceinline__ void rr_clear_edge0(RrXchg& X) {
  const int t = threadIdx.x;
  if (t < 2 * kRrRows) X.edge[0][t / kRrRows][t % kRrRows] = 0.0;
}

using RrVec = double[kRrRows];

// The segment's addresses are recomputed at every use (the empty asm hides
// the offset from common-subexpression elimination), so the addresses of the
// first load are not kept in registers across the whole solve.
__device__ __forceinline__ void rr_load(const double* G, const RrSeg& s, RrVec& v) {
  size_t off = s.off;
  asm volatile("" : "+v"(off));
#pragma unroll
  for (int e = 0; e < kRrRows; ++e) v[e] = e < s.nv ? G[off + (size_t)e * s.pitch] : 0.0;
}

__device__ __forceinline__ void rr_store(double* G, const RrSeg& s, const RrVec& v) {
  size_t off = s.off;
  asm volatile("" : "+v"(off));
#pragma unroll
  for (int e = 0; e < kRrRows; ++e)
    if (e < s.nv) G[off + (size_t)e * s.pitch] = v[e];
}

// After a transition: the state and the pass scalars back in scalar registers.
__device__ __forceinline__ void rr_uniform(State& st, Sc& sc) {
  st = uniform_state(st);
  sc.al = uniform(sc.al);
  sc.be = uniform(sc.be);
}

__device__ __forceinline__ void rr_publish(const RrVec& v, const RrSeg& s, RrXchg& X) {
  X.first[s.t] = v[0];
  X.last[s.t] = v[kRrRows - 1];
  if (s.lane == 0 || s.lane == kWave - 1) {
    double* d = X.edge[s.wave + 1][s.lane == 0 ? 0 : 1];
#pragma unroll
    for (int e = 0; e < kRrRows; ++e) d[e] = v[e];
  }
}

// Neighbour values of a published vector just outside this thread's segment:
// south of element 0 and north of element kRrRows-1 (from the segments below
// and above), and for lanes 0 / 63 the west / east neighbours from the
// adjacent wavefront.  `f` maps the published values to the vector the
// stencil is applied to (identity, or the classic direction update); X2 is a
// second published vector that f combines with the first.
template <class F>
struct RrHalo {
  double S, N;
  // the wavefront's west edge (used by lane 0) and east edge (used by lane
  // 63); wavefront-uniform addresses, so every lane reads the same entry
  const double *eW, *eE;
  const double *eW2, *eE2;
  F f;
};

template <class F>
__device__ __forceinline__ RrHalo<F> rr_halo(const RrSeg& s, const RrXchg& X, const RrXchg* X2,
                                             F f) {
  const int ts = s.south ? s.t - s.stride : s.t, tn = s.north ? s.t + s.stride : s.t;
  const double S = f(X.last[ts], X2 ? X2->last[ts] : 0.0);
  const double N = f(X.first[tn], X2 ? X2->first[tn] : 0.0);
  // west: lane 63 of the previous wavefront (the zero entry for wavefront 0);
  // east: lane 0 of the next (for the last wavefront an entry nobody uses)
  const int ww = s.wave, we = min(s.wave + 2, s.nw);
  return RrHalo<F>{s.south ? S : 0.0,
                   s.north ? N : 0.0,
                   X.edge[ww][1],
                   X.edge[we][0],
                   X2 ? X2->edge[ww][1] : nullptr,
                   X2 ? X2->edge[we][0] : nullptr,
                   f};
}

// (A v) at element e of the segment; zero for rows outside the grid.  vs is
// v[e-1] as it was before any update of this pass (the caller may have
// overwritten v[e-1] already); unused for e == 0.
template <class F>
__device__ __forceinline__ double rr_st5(const RrVec& v, double vs, const RrSeg& s,
                                         const RrHalo<F>& h, int e) {
  const double evW = h.f(h.eW[e], h.eW2 ? h.eW2[e] : 0.0);
  const double evE = h.f(h.eE[e], h.eE2 ? h.eE2[e] : 0.0);
  const double w = dpp<kDppWaveShr1>(v[e], evW);   // lane 0 keeps its west edge
  const double ea = dpp<kDppWaveShl1>(v[e], evE);  // lane 63 keeps its east edge
  const double so = e > 0 ? vs : h.S;
  const double no = e + 1 < kRrRows ? v[e + 1] : h.N;
  return e < s.nv ? st5(v[e], w, ea, so, no) : 0.0;
}

template <int D>
__device__ __forceinline__ void rr_publish_sums(const double* acc, const RrSeg& s,
                                                double (*tot)[2]) {
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double v = wave_sum_swz(acc[d]);
    if (s.lane == 0) tot[s.wave][d] = v;
  }
}

// Sums of the wavefront totals in wavefront order.  All kRrWaves entries are
// loaded at once (entries of absent wavefronts are read but not added).
template <int D>
__device__ __forceinline__ void rr_read_sums(const RrSeg& s, const double (*tot)[2],
                                             double* sum) {
  double2 t[kRrWaves];
#pragma unroll
  for (int w = 0; w < kRrWaves; ++w) t[w] = *reinterpret_cast<const double2*>(tot[w]);
  double v0 = t[0].x, v1 = t[0].y;
#pragma unroll
  for (int w = 1; w < kRrWaves; ++w) {
    const double a0 = v0 + t[w].x, a1 = v1 + t[w].y;
    v0 = w < s.nw ? a0 : v0;
    v1 = w < s.nw ? a1 : v1;
  }
  sum[0] = uniform(v0);
  if (D > 1) sum[1] = uniform(v1);
}

struct RrId {
  __device__ double operator()(double a, double) const { return a; }
};

// Classic direction update p = r + beta p_old (p = r on the first iteration).
struct RrDir {
  double be;
  bool first;
  __device__ double operator()(double rv, double pv) const {
    return first ? rv : fma(be, pv, rv);
  }
};

// true residual b - A x of the final iterate: slot (t,t); res2 = its sum
__device__ __forceinline__ void rr_final_residual(const PassArgs& a, const RrSeg& s, State& st,
                                                  const RrVec& x, RrXchg& X,
                                                  double (*tot_out)[2]) {
  rr_publish(x, s, X);
  __syncthreads();
  RrVec b;
  rr_load(a.b, s, b);
  const auto h = rr_halo(s, X, nullptr, RrId());
  double acc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < kRrRows; ++e) {
    const double t = b[e] - rr_st5(x, e > 0 ? x[e - 1] : 0.0, s, h, e);
    acc[0] = fma(t, t, acc[0]);
  }
  rr_publish_sums<1>(acc, s, tot_out);
  __syncthreads();
  double sum[1];
  rr_read_sums<1>(s, tot_out, sum);
  st.res2 = sum[0];
}

// One pass of Algorithm 2's loop (the K_PCG pass): sums of the previous
// pass, transition, then nvec = A w and the z, q, p, x, r, w recurrences with
// slots (r,r), (w,r).  FIRST: the first loop pass (z = nvec, q = w, p = r).
// Returns false when the solve stops.
template <bool FIRST>
__device__ __forceinline__ bool rr_pcg_pass(const RrSeg& s, RrLdsPcg& L, int& par, State& st,
                                            RrVec& r, RrVec& w, RrVec& p, RrVec& q, RrVec& z) {
  double sum[2];
  Sc sc;
  rr_read_sums<2>(s, L.tot[par], sum);
  if (!transition<K_PCG>(st, sum, sc)) return false;
  rr_uniform(st, sc);
  const double al = sc.al, be = sc.be, nal = -sc.al;
  const auto h = rr_halo(s, L.x[par], nullptr, RrId());
  double ac[2] = {0.0, 0.0};
  double wprev = 0.0;  // w[e-1] of this pass (w is updated in place)
#pragma unroll
  for (int e = 0; e < kRrRows; ++e) {
    const double nv = rr_st5(w, wprev, s, h, e);
    wprev = w[e];
    if (FIRST) {
      z[e] = nv;
      q[e] = w[e];
      p[e] = r[e];
    } else {
      z[e] = fma(be, z[e], nv);
      q[e] = fma(be, q[e], w[e]);
      p[e] = fma(be, p[e], r[e]);
    }
    L.xs[e][s.t] = fma(al, p[e], L.xs[e][s.t]);
    r[e] = fma(nal, q[e], r[e]);
    w[e] = fma(nal, z[e], w[e]);
    ac[0] = fma(r[e], r[e], ac[0]);
    ac[1] = fma(w[e], r[e], ac[1]);
  }
  par ^= 1;
  rr_publish(w, s, L.x[par]);
  rr_publish_sums<2>(ac, s, L.tot[par]);
  __syncthreads();
  return true;
}

// Pipelined CG (Algorithm 2) on one grid, x in LDS.
__device__ __forceinline__ void rr_solve_pcg(const PassArgs& a, State& st, char* raw) {
  RrLdsPcg& L = *reinterpret_cast<RrLdsPcg*>(raw);
  const RrSeg s = rr_seg(a.g);
  RrVec r, w, p, q, z;
  Sc sc;
  int par = 0;
  double sum[2] = {0.0, 0.0};
  rr_clear_edge0(L.x[0]);
  rr_clear_edge0(L.x[1]);
  {
    RrVec x;
    rr_load(a.x, s, x);
#pragma unroll
    for (int e = 0; e < kRrRows; ++e) L.xs[e][s.t] = x[e];
    rr_publish(x, s, L.x[par]);
    __syncthreads();
    // r = b - A x; slots (r,r), (b,b)
    transition<K_INIT_R>(st, sum, sc);
    RrVec b;
    rr_load(a.b, s, b);
    const auto h = rr_halo(s, L.x[par], nullptr, RrId());
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kRrRows; ++e) {
      r[e] = b[e] - rr_st5(x, e > 0 ? x[e - 1] : 0.0, s, h, e);
      acc[0] = fma(r[e], r[e], acc[0]);
      acc[1] = fma(b[e], b[e], acc[1]);
    }
    par ^= 1;
    rr_publish(r, s, L.x[par]);
    rr_publish_sums<2>(acc, s, L.tot[par]);
    __syncthreads();
  }
  rr_read_sums<2>(s, L.tot[par], sum);
  if (transition<K_INIT_W>(st, sum, sc)) {
    // w = A r; slots (r,r), (w,r)
    const auto h = rr_halo(s, L.x[par], nullptr, RrId());
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kRrRows; ++e) {
      w[e] = rr_st5(r, e > 0 ? r[e - 1] : 0.0, s, h, e);
      acc[0] = fma(r[e], r[e], acc[0]);
      acc[1] = fma(w[e], r[e], acc[1]);
    }
    par ^= 1;
    rr_publish(w, s, L.x[par]);
    rr_publish_sums<2>(acc, s, L.tot[par]);
    __syncthreads();
    bool go = rr_pcg_pass<true>(s, L, par, st, r, w, p, q, z);
    while (go) go = rr_pcg_pass<false>(s, L, par, st, r, w, p, q, z);
  }
  RrVec x;
#pragma unroll
  for (int e = 0; e < kRrRows; ++e) x[e] = L.xs[e][s.t];
  if (st.status != ST_ZERO_RHS) {
    par ^= 1;
    rr_final_residual(a, s, st, x, L.x[par], L.tot[par ^ 1]);
  }
  rr_store(a.x, s, x);
}

// Algorithm 1, first pass of an iteration (the K_CG1 pass): beta; p = r +
// beta p, also on the halo; s = A p; slot (p, s).  FIRST: p = r.
template <bool FIRST>
__device__ __forceinline__ bool rr_cg1_pass(const RrSeg& s, RrLdsCg& L, int& par, State& st,
                                            const RrVec& r, RrVec& p, RrVec& sv) {
  double sum[2];
  Sc sc;
  if (st.flags & F_BB_PENDING) rr_read_sums<2>(s, L.tot[par], sum);
  else rr_read_sums<1>(s, L.tot[par], sum);
  if (!transition<K_CG1>(st, sum, sc)) return false;
  rr_uniform(st, sc);
  const RrDir dir{sc.be, FIRST};
  const auto h = rr_halo(s, L.x[par][0], &L.x[par][1], dir);
  double acc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < kRrRows; ++e) p[e] = dir(r[e], p[e]);
#pragma unroll
  for (int e = 0; e < kRrRows; ++e) {
    sv[e] = rr_st5(p, e > 0 ? p[e - 1] : 0.0, s, h, e);
    acc[0] = fma(p[e], sv[e], acc[0]);
  }
  par ^= 1;
  rr_publish_sums<1>(acc, s, L.tot[par]);
  __syncthreads();
  return true;
}

// Algorithm 1, second pass (the K_CG2 pass): alpha; x += alpha p;
// r -= alpha s; slot (r, r).
__device__ __forceinline__ bool rr_cg2_pass(const RrSeg& s, RrLdsCg& L, int& par, State& st,
                                            RrVec& x, RrVec& r, const RrVec& p,
                                            const RrVec& sv) {
  double sum[1];
  Sc sc;
  rr_read_sums<1>(s, L.tot[par], sum);
  if (!transition<K_CG2>(st, sum, sc)) return false;
  rr_uniform(st, sc);
  const double al = sc.al, nal = -sc.al;
  double acc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < kRrRows; ++e) {
    x[e] = fma(al, p[e], x[e]);
    r[e] = fma(nal, sv[e], r[e]);
    acc[0] = fma(r[e], r[e], acc[0]);
  }
  par ^= 1;
  rr_publish(r, s, L.x[par][0]);
  rr_publish(p, s, L.x[par][1]);
  rr_publish_sums<1>(acc, s, L.tot[par]);
  __syncthreads();
  return true;
}

// Classic CG (Algorithm 1) on one grid, every vector in registers.
__device__ __forceinline__ void rr_solve_cg(const PassArgs& a, State& st, char* raw) {
  RrLdsCg& L = *reinterpret_cast<RrLdsCg*>(raw);
  const RrSeg s = rr_seg(a.g);
  RrVec x, r, p, sv;
  Sc sc;
  int par = 0;
  double sum[2] = {0.0, 0.0};
  rr_clear_edge0(L.x[0][0]);
  rr_clear_edge0(L.x[0][1]);
  rr_clear_edge0(L.x[1][0]);
  rr_clear_edge0(L.x[1][1]);
  rr_load(a.x, s, x);
  rr_publish(x, s, L.x[par][0]);
  __syncthreads();
  {
    // r = b - A x; slots (r,r), (b,b)
    transition<K_INIT_R>(st, sum, sc);
    RrVec b;
    rr_load(a.b, s, b);
    const auto h = rr_halo(s, L.x[par][0], nullptr, RrId());
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kRrRows; ++e) {
      r[e] = b[e] - rr_st5(x, e > 0 ? x[e - 1] : 0.0, s, h, e);
      acc[0] = fma(r[e], r[e], acc[0]);
      acc[1] = fma(b[e], b[e], acc[1]);
      p[e] = 0.0;
    }
    par ^= 1;
    rr_publish(r, s, L.x[par][0]);
    rr_publish(p, s, L.x[par][1]);
    rr_publish_sums<2>(acc, s, L.tot[par]);
    __syncthreads();
  }
  bool go = rr_cg1_pass<true>(s, L, par, st, r, p, sv) && rr_cg2_pass(s, L, par, st, x, r, p, sv);
  while (go)
    go = rr_cg1_pass<false>(s, L, par, st, r, p, sv) && rr_cg2_pass(s, L, par, st, x, r, p, sv);
  if (st.status != ST_ZERO_RHS) {
    par ^= 1;
    rr_final_residual(a, s, st, x, L.x[par][0], L.tot[par ^ 1]);
  }
  rr_store(a.x, s, x);
}

template <int VARIANT>
__global__ __launch_bounds__(kRrThreads) void k_solve_rr(PassArgs a) {
  __shared__ __attribute__((aligned(16))) char raw[kRrLdsBytes];
  State st = load_state_uniform(a.st_in);
  if constexpr (VARIANT == 1) rr_solve_pcg(a, st, raw);
  else rr_solve_cg(a, st, raw);
  if (threadIdx.x == 0) *a.st_out = st;
}

// Many register-resident solves, one per work-group: work-group i solves the
// resident solve in slot idx[i] (initial state in S[0]) and leaves its final
// state, marked done for the step engine, in both S[0] and S[1].  A wider
// work-group than the solve needs only adds idle wavefronts, whose zero sums
// leave every dot product unchanged.
__global__ __launch_bounds__(kRrThreads) void k_solve_rr_many(const Slot* slots,
                                                              const int* idx) {
  __shared__ __attribute__((aligned(16))) char raw[kRrLdsBytes];
  const Slot& S = slots[__builtin_amdgcn_readfirstlane(idx[blockIdx.x])];
  PassArgs a = {};
  a.g = S.g;
  a.b = S.b;
  a.x = S.x;
  State st = load_state_uniform(S.S[0]);
  if (S.variant == 1) rr_solve_pcg(a, st, raw);
  else rr_solve_cg(a, st, raw);
  st.kind = K_DONE;
  if (threadIdx.x == 0) {
    *S.S[0] = st;
    *S.S[1] = st;
  }
}

// ---------------------------------------------------- multi-solve step --
//
// One launch advances every resident solve by one pass.  The work is a table
// of items (tiles [t0, t1) of one solve); work-groups stride over it.  For
// each item a work-group reads its solve's state for this pass, sums the
// previous pass's tile partials, applies the transition of the pass kind the
// state names (exactly the prologue of a single-solve pass, hence the same
// bits), records the kind of the solve's next pass, and processes its tiles.
// The work-group holding tile 0 of a solve writes the solve's next state.
// Kernel boundaries order the steps: no atomics, no fences, no waiting.

template <int KIND>
__device__ __forceinline__ bool step_transition(State& s, const double* sum, Sc& sc) {
  if constexpr (KIND == K_FINAL) {
    sc.al = sc.be = sc.inv = sc.alp = 0.0;
    sc.first = 0;
    sc.xu = 0;
    s.res2 = sum[0];
    return false;
  } else {
    return transition<KIND>(s, sum, sc);
  }
}

// Kind of the pass after `kind`, given whether its body ran.  Preconditioned
// (precond != 0): classic CG runs K_CHEB, K_CG1, K_CG2 per iteration; the
// pipelined variant K_CHEB and K_INIT_WU once, then K_CHEBW, K_PPCG; the
// refinement's inner solve K_CHEBF, K_CG1F, K_CG2F.
__device__ __forceinline__ int next_kind(int kind, bool ran, const State& s, int variant,
                                         int refined, int precond, int rr_period = 0) {
  const int stop = s.status == ST_ZERO_RHS ? K_DONE : K_RESID;
  switch (kind) {
    case K_INIT_R:
      return precond ? K_CHEB : variant == 1 ? K_INIT_W : K_CG1;
    case K_INIT_W: return ran ? K_PCG : K_DONE;
    // residual replacement after every rr_period-th iteration (even, so x is
    // current): q = A p, z = A q, then r = b - A x and w = A r with their sums
    case K_PCG:
      return !ran ? stop : (rr_period > 0 && s.k % rr_period == 0) ? K_RRQ : K_PCG;
    case K_RRQ: return ran ? K_RRZ : stop;
    case K_RRZ: return ran ? K_INIT_R : stop;
    case K_CHEB: return ran ? (variant == 1 ? K_INIT_WU : K_CG1) : stop;
    case K_INIT_WU: return ran ? K_CHEBW : stop;
    case K_CHEBW: return ran ? K_PPCG : stop;
    case K_PPCG: return ran ? K_CHEBW : stop;
    case K_CG1: return ran ? K_CG2 : stop;
    case K_CG2: return ran ? (precond ? K_CHEB : K_CG1) : K_RESID;
    case K_RESID: return refined ? K_REF_SCALE : K_FINAL;
    case K_FINAL: return K_DONE;
    case K_REF_SCALE: return ran ? (precond ? K_CHEBF : K_CG1F) : K_DONE;
    case K_CHEBF: return ran ? K_CG1F : K_REF_UPDATE;
    case K_CG1F: return ran ? K_CG2F : K_REF_UPDATE;
    case K_CG2F: return ran ? (precond ? K_CHEBF : K_CG1F) : K_REF_UPDATE;
    case K_REF_UPDATE: return ran ? K_RESID : K_DONE;
  }
  return K_DONE;
}

// The pass arguments of a resident solve at pass m (vector ping-pong
// parities from the iteration counters k0, kin0 before the transition).
template <int KIND>
__device__ __forceinline__ PassArgs slot_args(const Slot& S, int m, int k0, int kin0) {
  PassArgs a;
  a.g = S.g;
  a.st_in = nullptr;
  a.st_out = nullptr;
  a.part_in = nullptr;
  a.part_out = S.part[(m + 1) & 1];
  a.b = S.b;
  a.x = S.x;
  // preconditioned classic pass 1 forms p = z + beta p
  a.r = (KIND == K_CG1 && S.precond) ? S.z : S.r;
  a.z = S.z;
  a.q = S.q;
  a.p = S.p;
  a.w_in = S.W[k0 & 1];
  a.w_out = (KIND == K_INIT_W) ? S.W[0] : S.W[(k0 + 1) & 1];
  a.pc_in = (KIND == K_CG2) ? S.PC[(k0 + 1) & 1] : S.PC[k0 & 1];
  a.pc_out = S.PC[(k0 + 1) & 1];
  a.pc_prev = S.PC[k0 & 1];
  // preconditioned inner pass 1 forms p = z + beta p
  a.rf = (KIND == K_CG1F && S.precond) ? S.zf : S.rf;
  a.df = S.df;
  a.zf = S.zf;
  a.pf_in = (KIND == K_CG2F) ? S.PF[(kin0 + 1) & 1] : S.PF[kin0 & 1];
  a.pf_out = S.PF[(kin0 + 1) & 1];
  a.pf_prev = S.PF[kin0 & 1];
  a.u = (KIND == K_RRQ) ? S.p : (KIND == K_RRZ) ? S.q : nullptr;
  a.y = (KIND == K_RRQ) ? S.q : (KIND == K_RRZ) ? S.z : nullptr;
  a.rev = 0;
  a.cheb_s = S.precond;
  a.cheb_rows = S.cheb_rows;
  a.cheb_tiles = S.cheb_tiles;
  a.cheb = S.cheb;
  a.uu = S.u;
  a.sv = S.sv;
  a.mv = S.mv;
  a.wv = S.W[0];
  return a;
}

template <int KIND, int CPL, int OP = 0>
__device__ __forceinline__ void step_item(const Slot& S, const Item& it, int m, State s,
                                          double* lds, int rev) {
  constexpr int DI = (KIND == K_FINAL) ? 1 : ndots_in<KIND>();
  constexpr int DO = (KIND == K_FINAL) ? 0 : ndots_out<KIND>();
  static_assert(DO <= 3, "at most three partial slots per pass");
  const int T = S.g.tiles;
  double sum[2] = {0.0, 0.0};
  if constexpr (DI > 0) {
    // classic pass 1 also takes (b,b) after the initial residual; with the
    // preconditioner its one slot is (r,z) in the Chebyshev pass's tiles
    const bool pc = (KIND == K_CG1 || KIND == K_CG1F) && (s.flags & F_PRECOND);
    const int din = (KIND == K_CG1) ? ((s.flags & F_BB_PENDING) && !pc ? 2 : 1) : DI;
    const int tin = pc ? S.cheb_tiles : T;
    if (s.status == ST_RUNNING || KIND == K_FINAL) {
      if (din == 2) cross_tile_sum<2>(S.part[m & 1], tin, sum, lds);
      else cross_tile_sum<1>(S.part[m & 1], tin, sum, lds);
    }
    sum[0] = uniform(sum[0]);
    sum[1] = uniform(sum[1]);
  }
  // ping-pong parities come from the iteration counters before the transition
  const int k0 = s.k, kin0 = s.kin;
  Sc sc;
  bool flush = false;
  bool run;
  if constexpr (KIND == K_FINAL) run = step_transition<KIND>(s, sum, sc);
  else run = transition_x<KIND>(s, sum, sc, flush);
  if (it.t0 == 0 && threadIdx.x == 0) {
    State o = s;
    o.kind = next_kind(KIND, run, s, S.variant, S.refined, S.precond, S.rr_period);
    *S.S[(m + 1) & 1] = o;
  }
  if (!run && !flush) return;
  const PassArgs a = slot_args<KIND>(S, m, k0, kin0);
  if constexpr (defers_x<KIND>()) {
    if (flush) {
      for (int t = it.t0; t < it.t1; ++t) run_flush<KIND, CPL>(a, t, sc);
      return;
    }
  }
  // odd steps walk the item's tiles backwards (see k_step)
  int par = 0;
  for (int tt = it.t0; tt < it.t1; ++tt, par ^= 1) {
    const int t = rev ? it.t1 - 1 - (tt - it.t0) : tt;
    double lv[3] = {0.0, 0.0, 0.0};
    if constexpr (KIND != K_FINAL) run_body_any<KIND, CPL, OP>(a, t, sc, lv);
    if constexpr (DO > 0) tile_partial<DO>(lv, a.part_out, T, t, lds + 8, par);
  }
}

// The operator of a resident solve: 0 the 5-point stencil, 1 the 7-point one
// (3D), 2 the variable-coefficient 5-point one.
__device__ __forceinline__ int slot_op(const Slot& S) {
  return S.g.plane > 0 ? 1 : S.g.kc ? 2 : 0;
}

// At least three waves per SIMD (168 VGPRs, no spill): its largest pass body
// would otherwise take 174 and two waves.
__global__ __launch_bounds__(kGroup, 3) void k_step(const Slot* slots, const Item* items,
                                                const int* n_items, const int* step_base,
                                                int k) {
  __shared__ double lds[kLdsPerGroup];
  const int n = __builtin_amdgcn_readfirstlane(*n_items);
  const int step = __builtin_amdgcn_readfirstlane(*step_base) + k;
  // odd steps take the items (and their tiles) in reverse order, so a step
  // starts on the tiles the previous one wrote last (memory-side cache)
  const int rev = step & 1;
  for (int ii = blockIdx.x; ii < n; ii += gridDim.x) {
    const Item it = items[rev ? n - 1 - ii : ii];
    const Slot& S = slots[__builtin_amdgcn_readfirstlane(it.slot)];
    // the 3D and variable-coefficient solves belong to k_step_op
    if (slot_op(S) != 0) continue;
    const int m = step - S.admit_step;
    const State s = load_state_uniform(S.S[m & 1]);
    const int kind = __builtin_amdgcn_readfirstlane(s.kind);
    if (kind == K_DONE) {
      if (it.t0 == 0 && threadIdx.x == 0) *S.S[(m + 1) & 1] = s;
      continue;
    }
    // the Chebyshev passes belong to the Chebyshev step kernel, the passes of
    // preconditioned pipelined CG to k_step_ppcg (their bodies would raise
    // this kernel's register count for every pass)
    if (kind == K_CHEB || kind == K_CHEBW || kind == K_CHEBF || kind == K_INIT_WU ||
        kind == K_PPCG)
      continue;
    if (S.cpl4) {
      switch (kind) {
        case K_INIT_R: step_item<K_INIT_R, 4>(S, it, m, s, lds, rev); break;
        case K_CG1: step_item<K_CG1, 4>(S, it, m, s, lds, rev); break;
        case K_CG2: step_item<K_CG2, 4>(S, it, m, s, lds, rev); break;
        case K_RESID: step_item<K_RESID, 4>(S, it, m, s, lds, rev); break;
        case K_FINAL: step_item<K_FINAL, 4>(S, it, m, s, lds, rev); break;
        case K_REF_SCALE: step_item<K_REF_SCALE, 4>(S, it, m, s, lds, rev); break;
        case K_CG1F: step_item<K_CG1F, 4>(S, it, m, s, lds, rev); break;
        case K_CG2F: step_item<K_CG2F, 4>(S, it, m, s, lds, rev); break;
        case K_REF_UPDATE: step_item<K_REF_UPDATE, 4>(S, it, m, s, lds, rev); break;
      }
    } else {
      switch (kind) {
        case K_INIT_R: step_item<K_INIT_R, 2>(S, it, m, s, lds, rev); break;
        case K_INIT_W: step_item<K_INIT_W, 2>(S, it, m, s, lds, rev); break;
        case K_PCG: step_item<K_PCG, 2>(S, it, m, s, lds, rev); break;
        case K_RRQ: step_item<K_RRQ, 2>(S, it, m, s, lds, rev); break;
        case K_RRZ: step_item<K_RRZ, 2>(S, it, m, s, lds, rev); break;
        case K_CG1: step_item<K_CG1, 2>(S, it, m, s, lds, rev); break;
        case K_CG2: step_item<K_CG2, 2>(S, it, m, s, lds, rev); break;
        case K_RESID: step_item<K_RESID, 2>(S, it, m, s, lds, rev); break;
        case K_FINAL: step_item<K_FINAL, 2>(S, it, m, s, lds, rev); break;
      }
    }
    __syncthreads();  // LDS reuse by the next item
  }
}

// Step *step_base + k of the resident solves on the operator OP (1: 3D
// 7-point, 2: variable coefficients; FP64 CG of either variant, no
// preconditioner), over the same items as k_step, which leaves them alone: a
// kernel of their own keeps their walkers' registers out of k_step.
// The 7-point form fits three waves per SIMD (168 VGPRs, no scratch); the
// variable-coefficient one would spill at three and keeps two (190 VGPRs).
template <int OP>
__global__ __launch_bounds__(kGroup, OP == 1 ? 3 : 2) void k_step_op(const Slot* slots,
                                                                      const Item* items,
                                                                      const int* n_items,
                                                                      const int* step_base,
                                                                      int k) {
  __shared__ double lds[kLdsPerGroup];
  const int n = __builtin_amdgcn_readfirstlane(*n_items);
  const int step = __builtin_amdgcn_readfirstlane(*step_base) + k;
  const int rev = step & 1;
  for (int ii = blockIdx.x; ii < n; ii += gridDim.x) {
    const Item it = items[rev ? n - 1 - ii : ii];
    const Slot& S = slots[__builtin_amdgcn_readfirstlane(it.slot)];
    if (slot_op(S) != OP) continue;
    const int m = step - S.admit_step;
    const State s = load_state_uniform(S.S[m & 1]);
    const int kind = __builtin_amdgcn_readfirstlane(s.kind);
    if (kind == K_DONE) {
      if (it.t0 == 0 && threadIdx.x == 0) *S.S[(m + 1) & 1] = s;
      continue;
    }
    switch (kind) {
      case K_INIT_R: step_item<K_INIT_R, 2, OP>(S, it, m, s, lds, rev); break;
      case K_INIT_W: step_item<K_INIT_W, 2, OP>(S, it, m, s, lds, rev); break;
      case K_PCG: step_item<K_PCG, 2, OP>(S, it, m, s, lds, rev); break;
      case K_RRQ: step_item<K_RRQ, 2, OP>(S, it, m, s, lds, rev); break;
      case K_RRZ: step_item<K_RRZ, 2, OP>(S, it, m, s, lds, rev); break;
      case K_CG1: step_item<K_CG1, 2, OP>(S, it, m, s, lds, rev); break;
      case K_CG2: step_item<K_CG2, 2, OP>(S, it, m, s, lds, rev); break;
      case K_RESID: step_item<K_RESID, 2, OP>(S, it, m, s, lds, rev); break;
      case K_FINAL: step_item<K_FINAL, 2, OP>(S, it, m, s, lds, rev); break;
    }
    __syncthreads();  // LDS reuse by the next item
  }
}

// The tile passes of preconditioned pipelined CG (K_INIT_WU, K_PPCG) at step
// *step_base + k, over the same items as k_step; every other pass kind is
// left to k_step and the Chebyshev step kernel.
__global__ __launch_bounds__(kGroup) void k_step_ppcg(const Slot* slots, const Item* items,
                                                     const int* n_items, const int* step_base,
                                                     int k) {
  __shared__ double lds[kLdsPerGroup];
  const int n = __builtin_amdgcn_readfirstlane(*n_items);
  const int step = __builtin_amdgcn_readfirstlane(*step_base) + k;
  const int rev = step & 1;
  for (int ii = blockIdx.x; ii < n; ii += gridDim.x) {
    const Item it = items[rev ? n - 1 - ii : ii];
    const Slot& S = slots[__builtin_amdgcn_readfirstlane(it.slot)];
    const int m = step - S.admit_step;
    const State s = load_state_uniform(S.S[m & 1]);
    const int kind = __builtin_amdgcn_readfirstlane(s.kind);
    if (kind == K_INIT_WU) step_item<K_INIT_WU, 2>(S, it, m, s, lds, rev);
    else if (kind == K_PPCG) step_item<K_PPCG, 2>(S, it, m, s, lds, rev);
    else continue;
    __syncthreads();  // LDS reuse by the next item
  }
}

// The Chebyshev passes of the step engine: for a solve whose state names
// K_CHEB or K_CHEBW (F32: K_CHEBF) at this step, the item's work-group sums
// the previous pass's partials, applies the transition of k_cheb (k_chebf)
// and marches Chebyshev items [t0, t1) of the solve exactly as k_cheb
// (k_chebf) does (same items, same partial tiles, hence the same bits); a
// stop after an odd iteration applies the pending x (d) update on the tiles
// matching the item's share instead.  Solves at any other pass are skipped
// (k_step and the other form of this kernel run them).  The binary32 form is
// a kernel of its own so that its march does not add to the registers of the
// binary64 one.
template <int S, bool F32>
__global__ __launch_bounds__(kChebThreads) void k_step_cheb(const Slot* slots, const Item* items,
                                                           const int* cinfo,
                                                           const int* step_base, int k) {
  __shared__ double colacc[kChebWaves * kChebOut];
  __shared__ double red[4 * 3];
  // this s's items: cinfo[2 s] items from items + cinfo[2 s + 1]
  const int n = __builtin_amdgcn_readfirstlane(cinfo[2 * S]);
  items += __builtin_amdgcn_readfirstlane(cinfo[2 * S + 1]);
  const int step = __builtin_amdgcn_readfirstlane(*step_base) + k;
  for (int ii = blockIdx.x; ii < n; ii += gridDim.x) {
    const Item it = items[ii];
    const Slot& Sl = slots[__builtin_amdgcn_readfirstlane(it.slot)];
    const int m = step - Sl.admit_step;
    State s = load_state_uniform(Sl.S[m & 1]);
    const int kind = __builtin_amdgcn_readfirstlane(s.kind);
    if (F32 ? kind != K_CHEBF : (kind != K_CHEB && kind != K_CHEBW)) continue;
    const bool pipe = kind == K_CHEBW;
    constexpr bool f32 = F32;
    const int T = Sl.g.tiles;
    double sum[3] = {0.0, 0.0, 0.0};
    if (s.status == ST_RUNNING) {
      if (pipe) cross_tile_sum<3>(Sl.part[m & 1], T, sum, red);
      else if (!f32 && (s.flags & F_BB_PENDING)) cross_tile_sum<2>(Sl.part[m & 1], T, sum, red);
      else cross_tile_sum<1>(Sl.part[m & 1], T, sum, red);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) sum[d] = uniform(sum[d]);
    const int k0 = s.k, kin0 = s.kin;
    Sc sc;
    bool flush = false;
    bool run;
    if constexpr (F32) run = transition_x<K_CHEBF>(s, sum, sc, flush);
    else run = pipe ? transition<K_CHEBW>(s, sum, sc) : transition_x<K_CHEB>(s, sum, sc, flush);
    if (it.t0 == 0 && threadIdx.x == 0) {
      State o = s;
      o.kind = next_kind(kind, run, s, Sl.variant, Sl.refined, Sl.precond);
      *Sl.S[(m + 1) & 1] = o;
    }
    PassArgs a = slot_args<K_CHEB>(Sl, m, k0, kin0);
    if (flush) {
      // the test stopped the solve after an odd iteration: x (d) update on
      // the tiles in proportion to this item's share of the Chebyshev items
      const int I = Sl.cheb_items;
      const int t0 = (int)((int64_t)T * it.t0 / I), t1 = (int)((int64_t)T * it.t1 / I);
      if (threadIdx.x < kGroup) {
        if constexpr (F32)
          for (int t = t0; t < t1; ++t) run_flush<K_CHEBF, 4>(a, t, sc);
        else
          for (int t = t0; t < t1; ++t) run_flush<K_CHEB, 2>(a, t, sc);
      }
      continue;
    }
    if (!run) continue;
    // input and output: classic z = M^-1 r; pipelined u = M^-1 r first, then
    // m = M^-1 w
    if (pipe) {
      a.r = Sl.W[0];
      a.z = Sl.mv;
    } else if (Sl.variant == 1) {
      a.z = Sl.u;
    }
    if constexpr (F32) {
      const int ngx = (cheb_ntx<float>(Sl.g) + kChebGroupTiles - 1) / kChebGroupTiles;
      for (int ci = it.t0; ci < it.t1; ++ci) cheb_item<S, false, float>(a, ci, ngx, colacc);
    } else {
      const int ngx = (Sl.g.ntx + kChebGroupTiles - 1) / kChebGroupTiles;
      for (int ci = it.t0; ci < it.t1; ++ci) {
        if (pipe) cheb_item<S, true>(a, ci, ngx, colacc);
        else cheb_item<S, false>(a, ci, ngx, colacc);
      }
    }
  }
}

__global__ void k_gather(const Slot* slots, const int* idx, int n, int step, State* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const Slot& S = slots[idx[i]];
    out[i] = *S.S[(step - S.admit_step) & 1];
  }
}

hipError_t launch_step(const Slot* slots, const Item* items, const int* n_items,
                       const int* step_base, int k, int grid, hipStream_t st) {
  if (grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_step, dim3(grid), dim3(kGroup), 0, st, slots, items, n_items, step_base,
                     k);
  return hipGetLastError();
}

hipError_t launch_step_ppcg(const Slot* slots, const Item* items, const int* n_items,
                            const int* step_base, int k, int grid, hipStream_t st) {
  if (grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_step_ppcg, dim3(grid), dim3(kGroup), 0, st, slots, items, n_items,
                     step_base, k);
  return hipGetLastError();
}

hipError_t launch_step_op(int op, const Slot* slots, const Item* items, const int* n_items,
                          const int* step_base, int k, int grid, hipStream_t st) {
  if (grid < 1 || (op != 1 && op != 2)) return hipErrorInvalidValue;
  if (op == 1)
    hipLaunchKernelGGL(k_step_op<1>, dim3(grid), dim3(kGroup), 0, st, slots, items, n_items,
                       step_base, k);
  else
    hipLaunchKernelGGL(k_step_op<2>, dim3(grid), dim3(kGroup), 0, st, slots, items, n_items,
                       step_base, k);
  return hipGetLastError();
}

int step_op_max_blocks_per_cu(int op) {
  int n = 0;
  const hipError_t e =
      op == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_op<1>, kGroup, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_op<2>, kGroup, 0);
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

int step_ppcg_max_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_ppcg, kGroup, 0) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int S>
static void launch_step_cheb_s(bool f32, const Slot* slots, const Item* items, const int* cinfo,
                               const int* step_base, int k, int grid, hipStream_t st) {
  if (f32)
    hipLaunchKernelGGL((k_step_cheb<S, true>), dim3(grid), dim3(kChebThreads), 0, st, slots,
                       items, cinfo, step_base, k);
  else
    hipLaunchKernelGGL((k_step_cheb<S, false>), dim3(grid), dim3(kChebThreads), 0, st, slots,
                       items, cinfo, step_base, k);
}

hipError_t launch_step_cheb(int s, bool f32, const Slot* slots, const Item* items,
                            const int* cinfo, const int* step_base, int k, int grid,
                            hipStream_t st) {
  if (grid < 1) return hipErrorInvalidValue;
  switch (s) {
    case 1: launch_step_cheb_s<1>(f32, slots, items, cinfo, step_base, k, grid, st); break;
    case 2: launch_step_cheb_s<2>(f32, slots, items, cinfo, step_base, k, grid, st); break;
    case 3: launch_step_cheb_s<3>(f32, slots, items, cinfo, step_base, k, grid, st); break;
    case 4: launch_step_cheb_s<4>(f32, slots, items, cinfo, step_base, k, grid, st); break;
    case 5: launch_step_cheb_s<5>(f32, slots, items, cinfo, step_base, k, grid, st); break;
    case 6: launch_step_cheb_s<6>(f32, slots, items, cinfo, step_base, k, grid, st); break;
    case 7: launch_step_cheb_s<7>(f32, slots, items, cinfo, step_base, k, grid, st); break;
    case 8: launch_step_cheb_s<8>(f32, slots, items, cinfo, step_base, k, grid, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather(const Slot* slots, const int* idx, int n, int step, State* out,
                         hipStream_t st) {
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((n + 63) / 64), dim3(64), 0, st, slots, idx, n, step, out);
  return hipGetLastError();
}

int step_max_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step, kGroup, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

// ------------------------------------------------------------ HBM probes --
//
// Plain streaming kernels over `nv` device vectors of n doubles (16 B per
// lane access, grid-stride): the attainable bandwidth of a read/write mix,
// and the copy kernel of known size that calibrates the traffic counters.
// pattern 0: read 1; 1: copy (1R 1W); 2: 2R 1W; 3: 3R 2W; 4: 6R 6W in place;
// 7: 6R 6W in place with the six vectors' rows interleaved (rows of 4096
// doubles, vector k's row j at (6 j + k) * 4096 of one block).
struct StreamArgs {
  double2* v[12];
  size_t n2;
  double* sink;
};

__device__ __forceinline__ void st_nt(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

template <int PATTERN>
__global__ __launch_bounds__(256) void k_stream(StreamArgs s) {
  double acc = 0.0;
  double2* const* v = s.v;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n2;
       i += (size_t)gridDim.x * blockDim.x) {
    if constexpr (PATTERN == 0) {
      const double2 a = v[0][i];
      acc += a.x + a.y;
    } else if constexpr (PATTERN == 1) {
      v[1][i] = v[0][i];
    } else if constexpr (PATTERN == 2) {
      const double2 a = v[0][i], b = v[1][i];
      v[2][i] = make_double2(a.x + 0.5 * b.x, a.y + 0.5 * b.y);
    } else if constexpr (PATTERN == 3) {
      const double2 a = v[0][i], b = v[1][i], c = v[2][i];
      v[3][i] = make_double2(a.x + b.x, a.y + b.y);
      v[4][i] = make_double2(b.x - c.x, b.y - c.y);
    } else if constexpr (PATTERN == 7) {
      constexpr size_t W2 = 2048;  // one row of 4096 doubles
      const size_t j = i / W2, c = i - j * W2;
      double2* r = v[0] + j * 6 * W2 + c;
      const double2 a = r[0], b = r[W2], cc = r[2 * W2], d = r[3 * W2], e = r[4 * W2],
                    f = r[5 * W2];
      r[0] = make_double2(a.x + 0.5 * b.x, a.y + 0.5 * b.y);
      r[W2] = make_double2(b.x - 0.25 * cc.x, b.y - 0.25 * cc.y);
      r[2 * W2] = make_double2(cc.x + d.x, cc.y + d.y);
      r[3 * W2] = make_double2(d.x * 0.75, d.y * 0.75);
      r[4 * W2] = make_double2(e.x + f.x, e.y + f.y);
      r[5 * W2] = make_double2(f.x - a.x, f.y - a.y);
    } else {
      // six vectors in; six out: in place (4), to six other vectors (5), or
      // in place with non-temporal stores (6)
      const double2 a = v[0][i], b = v[1][i], c = v[2][i], d = v[3][i], e = v[4][i], f = v[5][i];
      const double2 o[6] = {make_double2(a.x + 0.5 * b.x, a.y + 0.5 * b.y),
                            make_double2(b.x - 0.25 * c.x, b.y - 0.25 * c.y),
                            make_double2(c.x + d.x, c.y + d.y),
                            make_double2(d.x * 0.75, d.y * 0.75),
                            make_double2(e.x + f.x, e.y + f.y),
                            make_double2(f.x - a.x, f.y - a.y)};
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if constexpr (PATTERN == 5) v[6 + k][i] = o[k];
        else if constexpr (PATTERN == 6) st_nt(v[k] + i, o[k]);
        else v[k][i] = o[k];
      }
    }
  }
  if (PATTERN == 0 && acc == 1.2345678e300) s.sink[0] = acc;  // keeps the reads alive
}

hipError_t launch_stream(int pattern, double* const* v, size_t n, double* sink, int grid,
                         hipStream_t st) {
  StreamArgs s;
  for (int k = 0; k < 12; ++k) s.v[k] = (double2*)v[k];
  s.n2 = n / 2;
  s.sink = sink;
  switch (pattern) {
    case 0: hipLaunchKernelGGL(k_stream<0>, dim3(grid), dim3(256), 0, st, s); break;
    case 1: hipLaunchKernelGGL(k_stream<1>, dim3(grid), dim3(256), 0, st, s); break;
    case 2: hipLaunchKernelGGL(k_stream<2>, dim3(grid), dim3(256), 0, st, s); break;
    case 3: hipLaunchKernelGGL(k_stream<3>, dim3(grid), dim3(256), 0, st, s); break;
    case 4: hipLaunchKernelGGL(k_stream<4>, dim3(grid), dim3(256), 0, st, s); break;
    case 5: hipLaunchKernelGGL(k_stream<5>, dim3(grid), dim3(256), 0, st, s); break;
    case 6: hipLaunchKernelGGL(k_stream<6>, dim3(grid), dim3(256), 0, st, s); break;
    case 7:
      if (n % 4096) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_stream<7>, dim3(grid), dim3(256), 0, st, s);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers --

template <bool PIPE>
static hipError_t launch_cheb(const PassArgs& a, int grid, hipStream_t st) {
  const dim3 G(grid), B(kChebThreads);
  switch (a.cheb_s) {
    case 1: hipLaunchKernelGGL((k_cheb<1, PIPE>), G, B, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_cheb<2, PIPE>), G, B, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_cheb<3, PIPE>), G, B, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_cheb<4, PIPE>), G, B, 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_cheb<5, PIPE>), G, B, 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_cheb<6, PIPE>), G, B, 0, st, a); break;
    case 7: hipLaunchKernelGGL((k_cheb<7, PIPE>), G, B, 0, st, a); break;
    default: hipLaunchKernelGGL((k_cheb<8, PIPE>), G, B, 0, st, a); break;
  }
  return hipGetLastError();
}

static hipError_t launch_chebf(const PassArgs& a, int grid, hipStream_t st) {
  const dim3 G(grid), B(kChebThreads);
  switch (a.cheb_s) {
    case 1: hipLaunchKernelGGL((k_chebf<1>), G, B, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_chebf<2>), G, B, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_chebf<3>), G, B, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_chebf<4>), G, B, 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_chebf<5>), G, B, 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_chebf<6>), G, B, 0, st, a); break;
    case 7: hipLaunchKernelGGL((k_chebf<7>), G, B, 0, st, a); break;
    default: hipLaunchKernelGGL((k_chebf<8>), G, B, 0, st, a); break;
  }
  return hipGetLastError();
}

template <int KIND>
static hipError_t launch_kind(int fp32g, const PassArgs& a, int grid, hipStream_t st) {
  if (a.g.plane > 0 || a.g.kc) {
    // the 7-point or the variable-coefficient operator: FP64 geometry only
    if (fp32g || (a.g.plane > 0 && a.g.kc)) return hipErrorInvalidValue;
    if (a.g.plane > 0) hipLaunchKernelGGL((k_pass<KIND, 2, 1>), dim3(grid), dim3(kGroup), 0, st, a);
    else hipLaunchKernelGGL((k_pass<KIND, 2, 2>), dim3(grid), dim3(kGroup), 0, st, a);
  } else if (fp32g) {
    hipLaunchKernelGGL((k_pass<KIND, 4>), dim3(grid), dim3(kGroup), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_pass<KIND, 2>), dim3(grid), dim3(kGroup), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_pass(int kind, int fp32g, const PassArgs& a, int grid, hipStream_t st) {
  if (grid < 8 || (grid & 7)) return hipErrorInvalidValue;
  // 3D and variable-coefficient grids run the passes that launch_kind
  // dispatches, nothing else
  if ((a.g.plane > 0 || a.g.kc) && !(kind == K_INIT_R || kind == K_INIT_W || kind == K_PCG ||
                         kind == K_PCGX || kind == K_CG1 || kind == K_CG2 || kind == K_CG2X ||
                         kind == K_RESID || kind == K_APPLY || kind == K_DOT))
    return hipErrorInvalidValue;
  if (a.g.plane > 0 && (a.g.plane > a.g.ny || a.g.ny % a.g.plane)) return hipErrorInvalidValue;
  switch (kind) {
    case K_INIT_R: return launch_kind<K_INIT_R>(fp32g, a, grid, st);
    case K_INIT_W: return launch_kind<K_INIT_W>(fp32g, a, grid, st);
    case K_PCG: return launch_kind<K_PCG>(fp32g, a, grid, st);
    case K_PCGX: return launch_kind<K_PCGX>(fp32g, a, grid, st);
    case K_CG1: return launch_kind<K_CG1>(fp32g, a, grid, st);
    case K_CG2: return launch_kind<K_CG2>(fp32g, a, grid, st);
    case K_CG2X: return launch_kind<K_CG2X>(fp32g, a, grid, st);
    case K_RESID: return launch_kind<K_RESID>(fp32g, a, grid, st);
    case K_APPLY: return launch_kind<K_APPLY>(fp32g, a, grid, st);
    case K_DOT: return launch_kind<K_DOT>(fp32g, a, grid, st);
    case K_REF_SCALE:
      hipLaunchKernelGGL((k_pass<K_REF_SCALE, 4>), dim3(grid), dim3(kGroup), 0, st, a);
      return hipGetLastError();
    case K_CG1F:
      hipLaunchKernelGGL((k_pass<K_CG1F, 4>), dim3(grid), dim3(kGroup), 0, st, a);
      return hipGetLastError();
    case K_CG2FX:
      hipLaunchKernelGGL((k_pass<K_CG2FX, 4>), dim3(grid), dim3(kGroup), 0, st, a);
      return hipGetLastError();
    case K_CG2F:
      hipLaunchKernelGGL((k_pass<K_CG2F, 4>), dim3(grid), dim3(kGroup), 0, st, a);
      return hipGetLastError();
    case K_REF_UPDATE:
      hipLaunchKernelGGL((k_pass<K_REF_UPDATE, 4>), dim3(grid), dim3(kGroup), 0, st, a);
      return hipGetLastError();
    case K_CHEB:
      if (fp32g || a.cheb_s < 1 || a.cheb_s > kChebMaxSteps || !a.cheb || !a.z || !a.r ||
          a.cheb_rows < 1)
        return hipErrorInvalidValue;
      return launch_cheb<false>(a, grid, st);
    case K_CHEBW:
      if (fp32g || a.cheb_s < 1 || a.cheb_s > kChebMaxSteps || !a.cheb || !a.z || !a.r ||
          a.cheb_rows < 1)
        return hipErrorInvalidValue;
      return launch_cheb<true>(a, grid, st);
    case K_CHEBF:
      // FP32 geometry (4 columns per lane): the pending-update flush walks its tiles
      if (!fp32g || a.cheb_s < 1 || a.cheb_s > kChebMaxSteps || !a.cheb || !a.zf || !a.rf ||
          !a.df || !a.pf_in || a.cheb_rows < 1)
        return hipErrorInvalidValue;
      return launch_chebf(a, grid, st);
    case K_INIT_WU:
      if (fp32g || !a.uu || !a.wv || !a.r) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_pass<K_INIT_WU, 2>), dim3(grid), dim3(kGroup), 0, st, a);
      return hipGetLastError();
    case K_PPCG:
      if (fp32g || !a.uu || !a.wv || !a.mv || !a.sv || !a.r || !a.x || !a.z || !a.q || !a.p)
        return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_pass<K_PPCG, 2>), dim3(grid), dim3(kGroup), 0, st, a);
      return hipGetLastError();
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_final(const PassArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kGroup), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t st) {
  if (bytes & 3) return hipErrorInvalidValue;
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  const int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_solve_rr_many(const Slot* slots, const int* idx, int n, hipStream_t st) {
  if (n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_solve_rr_many, dim3(n), dim3(kRrThreads), 0, st, slots, idx);
  return hipGetLastError();
}

hipError_t launch_solve_rr(int variant, const PassArgs& a, int threads, hipStream_t st) {
  const int64_t need = (int64_t)(a.g.nx + 1) * ((a.g.ny + kRrRows - 1) / kRrRows);
  if (threads < kWave || threads > kRrThreads || threads % kWave || need > threads)
    return hipErrorInvalidValue;
  if (variant == 1) hipLaunchKernelGGL((k_solve_rr<1>), dim3(1), dim3(threads), 0, st, a);
  else hipLaunchKernelGGL((k_solve_rr<0>), dim3(1), dim3(threads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_solve_wg(int variant, const PassArgs& a, hipStream_t st) {
  if (variant == 1) hipLaunchKernelGGL((k_solve_wg<1>), dim3(1), dim3(kWgGroups * kGroup), 0, st, a);
  else hipLaunchKernelGGL((k_solve_wg<0>), dim3(1), dim3(kWgGroups * kGroup), 0, st, a);
  return hipGetLastError();
}

template <int KIND, int CPL>
static int occ() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pass<KIND, CPL>, kGroup, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int S>
static int occ_cheb(bool f32) {
  int n = 0;
  const hipError_t e =
      f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_chebf<S>, kChebThreads, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_cheb<S, false>, kChebThreads, 0);
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

int cheb_max_blocks_per_cu(int s, bool f32) {
  switch (s) {
    case 1: return occ_cheb<1>(f32);
    case 2: return occ_cheb<2>(f32);
    case 3: return occ_cheb<3>(f32);
    case 4: return occ_cheb<4>(f32);
    case 5: return occ_cheb<5>(f32);
    case 6: return occ_cheb<6>(f32);
    case 7: return occ_cheb<7>(f32);
    default: return occ_cheb<8>(f32);
  }
}

int pass_max_blocks_per_cu(int kind, int fp32g) {
  switch (kind) {
    case K_PCG:
    case K_PCGX: return fp32g ? occ<K_PCGX, 4>() : occ<K_PCGX, 2>();
    case K_PPCG: return occ<K_PPCG, 2>();
    case K_CG1: return fp32g ? occ<K_CG1, 4>() : occ<K_CG1, 2>();
    case K_CG2:
    case K_CG2X: return fp32g ? occ<K_CG2X, 4>() : occ<K_CG2X, 2>();
    case K_CG1F: return occ<K_CG1F, 4>();
    case K_CG2F:
    case K_CG2FX: return occ<K_CG2FX, 4>();
    default: return fp32g ? occ<K_RESID, 4>() : occ<K_RESID, 2>();
  }
}

// Algorithmic HBM bytes per unknown of each pass (each vector read or written
// once; halo re-reads are not counted).
size_t pass_algorithmic_bytes(int kind, int64_t dof) {
  size_t per = 0;
  switch (kind) {
    case K_INIT_R: per = 8 * 3; break;          // read x, b; write r
    case K_INIT_W: per = 8 * 2; break;          // read r; write w
    case K_PCG: per = 8 * 10; break;            // read r w p q z; write r w p q z
    case K_PCGX: per = 8 * 12; break;           // ... and read, write x
    case K_CG1: per = 8 * 3; break;             // read r, p_old; write p
    case K_CG2: per = 8 * 3; break;             // read p, r; write r
    case K_CG2X: per = 8 * 6; break;            // read p, p_prev, x, r; write x, r
    case K_RESID: per = 8 * 2; break;           // read x, b
    case K_REF_SCALE: per = 8 * 2 + 4 * 2; break;  // read x, b; write rho, d
    case K_CG1F: per = 4 * 3; break;             // read r, p_old; write p (FP32)
    case K_CG2F: per = 4 * 3; break;             // read p, r; write r
    case K_CG2FX: per = 4 * 6; break;            // read p, p_prev, d, r; write d, r
    case K_REF_UPDATE: per = 8 * 2 + 4; break;  // read x, d; write x
    case K_APPLY: per = 8 * 2; break;
    case K_DOT: per = 8 * 2; break;
    case K_CHEB: per = 8 * 2; break;            // read r; write z (halo not counted)
    case K_CHEBW: per = 8 * 2; break;           // read w; write m
    case K_CHEBF: per = 4 * 2; break;           // read r; write z (FP32)
    case K_INIT_WU: per = 8 * 3; break;         // read u, r; write w
    case K_PPCG: per = 8 * 17; break;           // read m x r u w z q s p; write all but m
  }
  return per * (size_t)dof;
}

}  // namespace cgk
