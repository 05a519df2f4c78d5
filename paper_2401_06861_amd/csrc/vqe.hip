// VQE energies and adjoint gradients for batches of parameter vectors.
//
// The VQE experiment of the paper (Sec. III, Fig. 4) evaluates
// E(theta) = <psi(theta)|H|psi(theta)> for a parametrised circuit.  Here the
// gradient is computed by adjoint differentiation (Jones & Gacon,
// arXiv:2009.02823): with phi = U_G...U_1|0>, lambda = H phi, E = Re<phi|lambda>,
// then for k = G..1:  g_k = Im<lambda|P_k|phi>  (for U_k = exp(-i theta P_k/2)),
// phi <- U_k^dag phi,  lambda <- U_k^dag lambda.
//
// Two execution paths share the op encoding:
//  * LDS-resident (n <= 12): one workgroup owns one theta vector and keeps
//    phi and lambda in LDS for the whole forward pass, H application and
//    backward sweep; a persistent grid walks the batch.  One launch per batch.
//  * Global (any n): one launch per gate over all B states (blockIdx.y = batch
//    element), phi and lambda in HBM, gradient partials per (state, gate, block)
//    reduced in a fixed order; the whole schedule is captured once per batch
//    size in a hipGraph and replayed.  With B = 1 and no graph this is the
//    plain per-circuit path.
// Every reduction has a fixed order that does not depend on B, so a theta
// vector gives bit-identical results alone or inside any batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "engine.h"

namespace nwq {

enum VqeKind { OP_ROT = 0, OP_RZZ = 1, OP_FIX1 = 2, OP_CX = 3, OP_CZ = 4, OP_SWAP = 5 };

struct VqeOp {
  int kind;
  int q0, q1;
  int param;   // theta index (OP_ROT, OP_RZZ), else -1
  int axis;    // OP_ROT: 0 X, 1 Y, 2 Z
  int slot;    // gradient slot (ordinal among parametrised ops), else -1
  int mat;     // OP_FIX1: index into the fixed-matrix table (8 double2: U then U^dag)
  int pad;
};

struct VqeTerm {
  unsigned long long x, z;
  double c;
  int y;       // popcount(x & z) mod 4
  int pad;
};

namespace {

typedef double vd2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned ins0(unsigned p, int q) { return ((p >> q) << (q + 1)) | (p & ((1u << q) - 1u)); }
__device__ __forceinline__ unsigned long long ins0l(unsigned long long p, int q) {
  return ((p >> q) << (q + 1)) | (p & ((1ull << q) - 1ull));
}
__device__ __forceinline__ vd2 mk(double a, double b) { vd2 r; r.x = a; r.y = b; return r; }
__device__ __forceinline__ vd2 cmul(vd2 a, vd2 b) { return mk(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)); }
__device__ __forceinline__ vd2 cfma(vd2 a, vd2 b, vd2 c) {
  return mk(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ vd2 ld(const double2* p) { return *reinterpret_cast<const vd2*>(p); }
__device__ __forceinline__ void st(double2* p, vd2 v) { *reinterpret_cast<vd2*>(p) = v; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over a full wave (all 64 lanes active) with DPP lane moves only, no LDS
// traffic: pairs within quads, quads (half mirror), half rows (mirror), then
// rows 0 -> 1 and 2 -> 3 (broadcast of lane 15) and rows 0..1 -> 3
// (broadcast of lane 31); lane 63 ends with the total, which every lane
// reads.  Lanes a move does not write add 0.  The order is fixed.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_full(double v) {
  v += dpp_move<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);        // row_half_mirror
  v += dpp_move<0x140>(v);        // row_mirror
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// 2x2 matrices.  Rotations exp(-i t P/2) are built branch-free (the axis
// picks entries with selects) and fixed gates are loaded from the table in
// separate code paths: with this toolchain a branchy construction of the
// rotation matrix whose results merged with the table load was compiled to
// code that dropped the imaginary part of the RZ diagonal, so the two cases
// are never merged into one value.  The adjoint of a rotation is the
// rotation by -t.
struct M2 { vd2 m0, m1, m2, m3; };

__device__ __forceinline__ M2 rot_matrix(int axis, double theta, bool dag) {
  double s, c;
  sincos(0.5 * theta, &s, &c);
  s = dag ? -s : s;
  const double z = 0.0;
  M2 r;
  r.m0 = mk(c, axis == 2 ? -s : z);
  r.m1 = mk(axis == 1 ? -s : z, axis == 0 ? -s : z);
  r.m2 = mk(axis == 1 ? s : z, axis == 0 ? -s : z);
  r.m3 = mk(c, axis == 2 ? s : z);
  return r;
}

__device__ __forceinline__ M2 fixed_matrix(int mat, const double2* fixed, bool dag) {
  const double2* f = fixed + 8 * mat + (dag ? 4 : 0);
  M2 r;
  r.m0 = ld(f); r.m1 = ld(f + 1); r.m2 = ld(f + 2); r.m3 = ld(f + 3);
  return r;
}

// RZZ: diagonal e^{-i t/2} (even parity), e^{+i t/2} (odd parity)
__device__ __forceinline__ void rzz_phases(double theta, bool dag, vd2& even, vd2& odd) {
  double s, c;
  sincos(0.5 * theta, &s, &c);
  s = dag ? -s : s;
  even = mk(c, -s);
  odd = mk(c, s);
}

template <typename Idx>
__device__ __forceinline__ void pairs_apply(double2* v, Idx N, int q, const M2& m, Idx tid, Idx nt) {
  const Idx off = Idx(1) << q;
  for (Idx p = tid; p < (N >> 1); p += nt) {
    const Idx i0 = ((p >> q) << (q + 1)) | (p & (off - 1));
    const vd2 a = ld(v + i0), b = ld(v + i0 + off);
    st(v + i0, cfma(m.m0, a, cmul(m.m1, b)));
    st(v + i0 + off, cfma(m.m2, a, cmul(m.m3, b)));
  }
}

// Contribution Im( conj(l0) (P phi)_0 + conj(l1) (P phi)_1 ) of one pair for a
// single-qubit Pauli generator on the pair's qubit, written with scalar
// selects only (no per-axis branches building vectors; see rot_matrix):
//   X: Im(conj(l0) p1) + Im(conj(l1) p0)
//   Y: Re(conj(l1) p0) - Re(conj(l0) p1)        ((Y phi)_0 = -i p1, (Y phi)_1 = i p0)
//   Z: Im(conj(l0) p0) - Im(conj(l1) p1)
__device__ __forceinline__ double pair_grad(int axis, vd2 p0, vd2 p1, vd2 l0, vd2 l1) {
  const double im01 = l0.x * p1.y - l0.y * p1.x;
  const double im10 = l1.x * p0.y - l1.y * p0.x;
  const double re01 = l0.x * p1.x + l0.y * p1.y;
  const double re10 = l1.x * p0.x + l1.y * p0.y;
  const double im00 = l0.x * p0.y - l0.y * p0.x;
  const double im11 = l1.x * p1.y - l1.y * p1.x;
  const double gx = im01 + im10, gy = re10 - re01, gz = im00 - im11;
  return axis == 0 ? gx : (axis == 1 ? gy : gz);
}

// ---------------------------------------------------------------------------
// Gate application on one state held in LDS (or in global memory for the
// per-gate path: same code, different pointer).  Threads tid..nt stride.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void apply_op_state(double2* v, int n, const VqeOp& op, const double* th, const double2* fixed, bool dag,
                               unsigned tid, unsigned nt) {
  const unsigned N = 1u << n;
  switch (op.kind) {
    case OP_ROT:
      pairs_apply<unsigned>(v, N, op.q0, rot_matrix(op.axis, th[op.param], dag), tid, nt);
      break;
    case OP_FIX1:
      pairs_apply<unsigned>(v, N, op.q0, fixed_matrix(op.mat, fixed, dag), tid, nt);
      break;
    case OP_RZZ: {
      vd2 e, o;
      rzz_phases(th[op.param], dag, e, o);
      for (unsigned j = tid; j < N; j += nt) {
        const unsigned par = ((j >> op.q0) ^ (j >> op.q1)) & 1u;
        st(v + j, cmul(par ? o : e, ld(v + j)));
      }
      break;
    }
    case OP_CZ: {
      for (unsigned j = tid; j < N; j += nt)
        if (((j >> op.q0) & (j >> op.q1)) & 1u) { const vd2 x = ld(v + j); st(v + j, mk(-x.x, -x.y)); }
      break;
    }
    default: {   // OP_CX (control q0, target q1) or OP_SWAP: exchange two members of each quad
      const int lo = min(op.q0, op.q1), hi = max(op.q0, op.q1);
      const unsigned oa = op.kind == OP_CX ? (1u << op.q0) : (1u << op.q0);
      const unsigned ob = op.kind == OP_CX ? (1u << op.q0) + (1u << op.q1) : (1u << op.q1);
      for (unsigned p = tid; p < (N >> 2); p += nt) {
        const unsigned b = ins0(ins0(p, lo), hi);
        const vd2 x = ld(v + b + oa), y = ld(v + b + ob);
        st(v + b + oa, y);
        st(v + b + ob, x);
      }
      break;
    }
  }
}

// One backward step on (phi, lam): returns this thread's gradient partial
// (0 for unparametrised ops) and applies U^dag to both states.
__device__ __forceinline__ double adjoint_step(double2* phi, double2* lam, int n, const VqeOp& op, const double* th,
                               const double2* fixed, unsigned tid, unsigned nt) {
  const unsigned N = 1u << n;
  double g = 0.0;
  if (op.kind == OP_ROT) {
    const M2 m = rot_matrix(op.axis, th[op.param], true);
    const unsigned off = 1u << op.q0;
    for (unsigned p = tid; p < (N >> 1); p += nt) {
      const unsigned i0 = ins0(p, op.q0);
      const vd2 p0 = ld(phi + i0), p1 = ld(phi + i0 + off);
      const vd2 l0 = ld(lam + i0), l1 = ld(lam + i0 + off);
      g += pair_grad(op.axis, p0, p1, l0, l1);
      st(phi + i0, cfma(m.m0, p0, cmul(m.m1, p1)));
      st(phi + i0 + off, cfma(m.m2, p0, cmul(m.m3, p1)));
      st(lam + i0, cfma(m.m0, l0, cmul(m.m1, l1)));
      st(lam + i0 + off, cfma(m.m2, l0, cmul(m.m3, l1)));
    }
  } else if (op.kind == OP_RZZ) {
    vd2 e, o;
    rzz_phases(th[op.param], true, e, o);
    for (unsigned j = tid; j < N; j += nt) {
      const unsigned par = ((j >> op.q0) ^ (j >> op.q1)) & 1u;
      const vd2 p = ld(phi + j), l = ld(lam + j);
      const double t = l.x * p.y - l.y * p.x;   // Im(conj(l) p), generator Z Z = +-1
      g += par ? -t : t;
      st(phi + j, cmul(par ? o : e, p));
      st(lam + j, cmul(par ? o : e, l));
    }
  } else {
    apply_op_state(phi, n, op, th, fixed, true, tid, nt);
    apply_op_state(lam, n, op, th, fixed, true, tid, nt);
  }
  return g;
}

// (H phi)_j = sum_t c_t i^y (-1)^{|(j^x)&z|} phi_{j^x}
__device__ __forceinline__ vd2 h_apply_at(const double2* phi, unsigned long long j, const VqeTerm* terms, int nterms,
                                          const double* cb) {
  vd2 acc = mk(0.0, 0.0);
  for (int t = 0; t < nterms; ++t) {
    const VqeTerm T = terms[t];
    const double tc = cb ? cb[t] : T.c;
    const unsigned long long k = j ^ T.x;
    vd2 v = ld(phi + k);
    switch (T.y & 3) {
      case 1: v = mk(-v.y, v.x); break;
      case 2: v = mk(-v.x, -v.y); break;
      case 3: v = mk(v.y, -v.x); break;
      default: break;
    }
    const double c = (__popcll(k & T.z) & 1) ? -tc : tc;
    acc.x = fma(c, v.x, acc.x);
    acc.y = fma(c, v.y, acc.y);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// LDS-resident persistent kernel (n <= 12)
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_vqe_lds(int n, const VqeOp* __restrict__ ops, int nops,
                                                const double2* __restrict__ fixed, const VqeTerm* __restrict__ terms,
                                                int nterms, int nslots, const int* __restrict__ slot_param,
                                                const double* __restrict__ theta, int P, int B,
                                                const double* __restrict__ coeffs,
                                                double* __restrict__ E, double* __restrict__ grad) {
  extern __shared__ double2 lds[];
  constexpr int NW = NT / kWave;
  const unsigned N = 1u << n;
  double2* phi = lds;
  double2* lam = lds + N;
  double* red = reinterpret_cast<double*>(grad ? lds + 2 * N : lds + N);   // [NW] scratch
  double* gpart = red + NW;                                              // [nslots][NW]
  const unsigned tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const double* th = theta + (size_t)b * P;
    __syncthreads();
    for (unsigned j = tid; j < N; j += NT) phi[j] = make_double2(j == 0 ? 1.0 : 0.0, 0.0);
    __syncthreads();
    for (int i = 0; i < nops; ++i) {
      apply_op_state(phi, n, ops[i], th, fixed, false, tid, NT);
      __syncthreads();
    }
    // lambda = H phi and E = Re <phi|lambda>
    double e = 0.0;
    for (unsigned j = tid; j < N; j += NT) {
      const vd2 l = h_apply_at(phi, j, terms, nterms, coeffs ? coeffs + (size_t)b * nterms : nullptr);
      const vd2 p = ld(phi + j);
      e += p.x * l.x + p.y * l.y;
      if (grad) st(lam + j, l);
    }
    e = wave_sum(e);
    if (lane == 0) red[wave] = e;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += red[w];
      E[b] = s;
    }
    if (!grad) continue;
    for (int i = nops - 1; i >= 0; --i) {
      const VqeOp op = ops[i];
      const double g = adjoint_step(phi, lam, n, op, th, fixed, tid, NT);
      if (op.slot >= 0) {
        const double w = wave_sum(g);
        if (lane == 0) gpart[op.slot * NW + wave] = w;
      }
      __syncthreads();
    }
    // grad[b][p] = sum over the slots of p (slot order) of the wave partials (wave order)
    if (tid == 0) {
      for (int p = 0; p < P; ++p) grad[(size_t)b * P + p] = 0.0;
      for (int s = 0; s < nslots; ++s) {
        double v = 0.0;
        for (int w = 0; w < NW; ++w) v += gpart[s * NW + w];
        grad[(size_t)b * P + slot_param[s]] += v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Global per-gate kernels: grid (blocks per state, B)
// ---------------------------------------------------------------------------
constexpr int kVqeBlock = 256;

__global__ __launch_bounds__(kVqeBlock) void k_vqe_init(double2* __restrict__ phi, int n) {
  const unsigned long long N = 1ull << n;
  double2* v = phi + (size_t)blockIdx.y * N;
  for (unsigned long long j = (unsigned long long)blockIdx.x * kVqeBlock + threadIdx.x; j < N;
       j += (unsigned long long)gridDim.x * kVqeBlock)
    v[j] = make_double2(j == 0 ? 1.0 : 0.0, 0.0);
}

// Grid-stride loops of the per-gate kernels take kU groups per thread per
// step, all loads issued before the arithmetic; the tail takes one.
constexpr int kU = 4;

__device__ __forceinline__ void pairs_apply_g(double2* v, unsigned long long N, int q, const M2& m,
                                              unsigned long long tid, unsigned long long nt) {
  const unsigned long long off = 1ull << q, np = N >> 1;
  unsigned long long p = tid;
  for (; p + (kU - 1) * nt < np; p += kU * nt) {
    unsigned long long i0[kU];
    vd2 a[kU], b[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      i0[u] = ins0l(p + u * nt, q);
      a[u] = ld(v + i0[u]);
      b[u] = ld(v + i0[u] + off);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      st(v + i0[u], cfma(m.m0, a[u], cmul(m.m1, b[u])));
      st(v + i0[u] + off, cfma(m.m2, a[u], cmul(m.m3, b[u])));
    }
  }
  for (; p < np; p += nt) {
    const unsigned long long i0 = ins0l(p, q);
    const vd2 a = ld(v + i0), b = ld(v + i0 + off);
    st(v + i0, cfma(m.m0, a, cmul(m.m1, b)));
    st(v + i0 + off, cfma(m.m2, a, cmul(m.m3, b)));
  }
}

__global__ __launch_bounds__(kVqeBlock) void k_vqe_gate(double2* __restrict__ states, int n, VqeOp op,
                                                        const double2* __restrict__ fixed,
                                                        const double* __restrict__ theta, int P, int dag) {
  const unsigned long long N = 1ull << n;
  double2* v = states + (size_t)blockIdx.y * N;
  const double* th = theta + (size_t)blockIdx.y * P;
  const unsigned long long tid = (unsigned long long)blockIdx.x * kVqeBlock + threadIdx.x;
  const unsigned long long nt = (unsigned long long)gridDim.x * kVqeBlock;
  switch (op.kind) {
    case OP_ROT:
      pairs_apply_g(v, N, op.q0, rot_matrix(op.axis, th[op.param], dag != 0), tid, nt);
      break;
    case OP_FIX1:
      pairs_apply_g(v, N, op.q0, fixed_matrix(op.mat, fixed, dag != 0), tid, nt);
      break;
    case OP_RZZ: {
      vd2 e, o;
      rzz_phases(th[op.param], dag != 0, e, o);
      unsigned long long j = tid;
      for (; j + (kU - 1) * nt < N; j += kU * nt) {
        vd2 x[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) x[u] = ld(v + j + u * nt);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const unsigned long long i = j + u * nt;
          const unsigned par = (unsigned)(((i >> op.q0) ^ (i >> op.q1)) & 1ull);
          st(v + i, cmul(par ? o : e, x[u]));
        }
      }
      for (; j < N; j += nt) {
        const unsigned par = (unsigned)(((j >> op.q0) ^ (j >> op.q1)) & 1ull);
        st(v + j, cmul(par ? o : e, ld(v + j)));
      }
      break;
    }
    case OP_CZ: {   // negate the quarter with both bits set
      const int lo = min(op.q0, op.q1), hi = max(op.q0, op.q1);
      const unsigned long long o11 = (1ull << op.q0) + (1ull << op.q1);
      for (unsigned long long p = tid; p < (N >> 2); p += nt) {
        const unsigned long long i = ins0l(ins0l(p, lo), hi) + o11;
        const vd2 x = ld(v + i);
        st(v + i, mk(-x.x, -x.y));
      }
      break;
    }
    default: {
      const int lo = min(op.q0, op.q1), hi = max(op.q0, op.q1);
      const unsigned long long oa = 1ull << op.q0;
      const unsigned long long ob = op.kind == OP_CX ? (1ull << op.q0) + (1ull << op.q1) : (1ull << op.q1);
      const unsigned long long nq = N >> 2;
      unsigned long long p = tid;
      for (; p + (kU - 1) * nt < nq; p += kU * nt) {
        unsigned long long b[kU];
        vd2 x[kU], y[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          b[u] = ins0l(ins0l(p + u * nt, lo), hi);
          x[u] = ld(v + b[u] + oa);
          y[u] = ld(v + b[u] + ob);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          st(v + b[u] + oa, y[u]);
          st(v + b[u] + ob, x[u]);
        }
      }
      for (; p < nq; p += nt) {
        const unsigned long long b = ins0l(ins0l(p, lo), hi);
        const vd2 x = ld(v + b + oa), y = ld(v + b + ob);
        st(v + b + oa, y);
        st(v + b + ob, x);
      }
      break;
    }
  }
}

// lambda = H phi, energy partials epart[b * G + block]
__global__ __launch_bounds__(kVqeBlock) void k_vqe_hphi(const double2* __restrict__ phi, double2* __restrict__ lam,
                                                        int n, const VqeTerm* __restrict__ terms, int nterms,
                                                        const double* __restrict__ coeffs,
                                                        double* __restrict__ epart, int store_lam) {
  __shared__ double red[kVqeBlock / kWave];
  const unsigned long long N = 1ull << n;
  const double2* p = phi + (size_t)blockIdx.y * N;
  double2* l = lam + (size_t)blockIdx.y * N;
  double e = 0.0;
  for (unsigned long long j = (unsigned long long)blockIdx.x * kVqeBlock + threadIdx.x; j < N;
       j += (unsigned long long)gridDim.x * kVqeBlock) {
    const vd2 h = h_apply_at(p, j, terms, nterms, coeffs ? coeffs + (size_t)blockIdx.y * nterms : nullptr);
    const vd2 v = ld(p + j);
    e += v.x * h.x + v.y * h.y;
    if (store_lam) st(l + j, h);
  }
  e = wave_sum(e);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kVqeBlock / kWave; ++w) s += red[w];
    epart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// lambda = H phi over tiles staged in LDS (fused schedule).  A pass takes a
// tile shape (low c bits plus m high bits) and the terms whose flipped bits
// x lie inside it; the first pass also takes every diagonal term (x = 0) and
// writes lambda, later passes add to it.  For entry j of a tile (local index
// l) a term contributes c_t i^y (-1)^{|(j ^ x) & z|} phi[j ^ x], with the
// partner read from the tile; the sign splits into the tile-local bits
// (|(l ^ xl) & zl|) and a per-tile constant (|base & zo| + |x & z|, on the
// bits outside the tile).  The last pass also sums Re<phi|lambda> into the
// energy partial of its workgroup.  Terms whose flipped bits fit no tile
// take a gather pass of their own (k_vqe_hphi_wide).
// ---------------------------------------------------------------------------
constexpr int kHBlock = 1024;     // threads per tile workgroup
constexpr int kHTileBits = 13;    // tiles of at most 2^13 entries (128 KiB of LDS)
constexpr int kHPer = (1 << kHTileBits) / kHBlock;
constexpr int kHMaxTerms = 128;   // terms per launch

struct HTerm {
  unsigned xl, zl;            // x and the z bits inside the tile, tile-local
  unsigned long long zo;      // z bits outside the tile (global)
  int y;                      // popcount(x & z) mod 4 (the i^y factor)
  int sx;                     // popcount(x & z) mod 2 (the sign of (j ^ x) vs j)
  int t;                      // index of the term (its coefficient)
  int pad;
};
struct HPass {
  int c, m;
  int hi[8];
  int first, last;
  int t_begin, n_diag, n_flip;   // diagonal terms first, then flipped ones
  int pad;
};

__host__ __device__ inline unsigned hpad(unsigned l) { return l + (l >> 4); }

template <bool FIRST, bool LAST>
__global__ __launch_bounds__(kHBlock) void k_vqe_hphi_tile(const double2* __restrict__ phi0, double2* __restrict__ lam0,
                                                           int n, HPass ps, const HTerm* __restrict__ hterms,
                                                           const VqeTerm* __restrict__ terms, int nterms,
                                                           const double* __restrict__ coeffs,
                                                           double* __restrict__ epart) {
  extern __shared__ double2 tl[];
  __shared__ double s_c[kHMaxTerms];
  __shared__ double red[kHBlock / kWave];
  const unsigned long long N = 1ull << n;
  const double2* __restrict__ phi = phi0 + (size_t)blockIdx.y * N;
  double2* __restrict__ lam = lam0 + (size_t)blockIdx.y * N;
  const int k = ps.c + ps.m;
  const unsigned len = 1u << k;
  const unsigned long long ntiles = 1ull << (n - k);
  const unsigned tid = threadIdx.x;
  const int nt = ps.n_diag + ps.n_flip;
  for (int i = tid; i < nt; i += kHBlock) {
    const int t = hterms[ps.t_begin + i].t;
    s_c[i] = coeffs ? coeffs[(size_t)blockIdx.y * nterms + t] : terms[t].c;
  }
  // Entry r of this thread is tile entry l = tid + r kHBlock; its global
  // index is the tile base plus a tile-independent part, computed once.
  const unsigned cmask = (1u << ps.c) - 1u;
  unsigned long long sc[kHPer];
#pragma unroll
  for (int r = 0; r < kHPer; ++r) {
    const unsigned l = tid + r * kHBlock;
    unsigned long long gi = l & cmask;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < ps.m && ((l >> (ps.c + i)) & 1u)) gi |= 1ull << ps.hi[i];
    sc[r] = gi;
  }
  double e = 0.0;
  for (unsigned long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    unsigned long long base = tile << ps.c;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < ps.m) {
        const int q = ps.hi[i];
        base = ((base >> q) << (q + 1)) | (base & ((1ull << q) - 1ull));
      }
    }
    vd2 v[kHPer], acc[kHPer];
    __syncthreads();   // the previous tile's readers are done (and s_c is written)
#pragma unroll
    for (int r = 0; r < kHPer; ++r) {
      const unsigned l = tid + r * kHBlock;
      if (l < len) {
        v[r] = __builtin_nontemporal_load(reinterpret_cast<const vd2*>(phi + (base | sc[r])));
        acc[r] = FIRST ? mk(0.0, 0.0) : __builtin_nontemporal_load(reinterpret_cast<const vd2*>(lam + (base | sc[r])));
        st(tl + hpad(l), v[r]);
      }
    }
    __syncthreads();
    // The sign of a term at entry l: the parity of (l & zl) splits into the
    // thread's bits (tid & zl) and the entry slot's (r kHBlock & zl); the bits
    // outside the tile (base & zo) and x & z are per tile and term.
    if (ps.n_diag > 0) {
      double d[kHPer];
#pragma unroll
      for (int r = 0; r < kHPer; ++r) d[r] = 0.0;
      for (int i = 0; i < ps.n_diag; ++i) {
        const HTerm T = hterms[ps.t_begin + i];
        const double c = s_c[i];
        const unsigned pb = (unsigned)(__popcll(base & T.zo) + __popc(tid & T.zl)) & 1u;
#pragma unroll
        for (int r = 0; r < kHPer; ++r) {
          const unsigned sg = pb ^ ((unsigned)__popc((unsigned)(r * kHBlock) & T.zl) & 1u);
          d[r] += sg ? -c : c;
        }
      }
#pragma unroll
      for (int r = 0; r < kHPer; ++r) {
        acc[r].x = fma(d[r], v[r].x, acc[r].x);
        acc[r].y = fma(d[r], v[r].y, acc[r].y);
      }
    }
    for (int i = ps.n_diag; i < nt; ++i) {
      const HTerm T = hterms[ps.t_begin + i];
      const double c = s_c[i];
      const unsigned pb = (unsigned)(__popcll(base & T.zo) + __popc(tid & T.zl) + T.sx) & 1u;
      const int y = T.y & 3;
#pragma unroll
      for (int r = 0; r < kHPer; ++r) {
        const unsigned l = tid + r * kHBlock;
        if (l >= len) continue;
        vd2 p = ld(tl + hpad(l ^ T.xl));
        if (y == 1) p = mk(-p.y, p.x);
        else if (y == 2) p = mk(-p.x, -p.y);
        else if (y == 3) p = mk(p.y, -p.x);
        const unsigned sg = pb ^ ((unsigned)__popc((unsigned)(r * kHBlock) & T.zl) & 1u);
        const double cf = sg ? -c : c;
        acc[r].x = fma(cf, p.x, acc[r].x);
        acc[r].y = fma(cf, p.y, acc[r].y);
      }
    }
#pragma unroll
    for (int r = 0; r < kHPer; ++r) {
      const unsigned l = tid + r * kHBlock;
      if (l >= len) continue;
      __builtin_nontemporal_store(acc[r], reinterpret_cast<vd2*>(lam + (base | sc[r])));
      if (LAST) e += v[r].x * acc[r].x + v[r].y * acc[r].y;
    }
  }
  if (LAST) {
    e = wave_sum_full(e);
    if ((tid & (kWave - 1)) == 0) red[tid / kWave] = e;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kHBlock / kWave; ++w) s += red[w];
      epart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
  }
}

// Terms whose flipped bits span more high bits than a tile holds: partners
// gathered from global memory (as k_vqe_hphi), added to lambda (written on
// the first pass); the last pass also sums the energy partials.
template <bool FIRST, bool LAST>
__global__ __launch_bounds__(kVqeBlock) void k_vqe_hphi_wide(const double2* __restrict__ phi0, double2* __restrict__ lam0,
                                                             int n, const VqeTerm* __restrict__ terms,
                                                             const int* __restrict__ tidx, int cnt, int nterms,
                                                             const double* __restrict__ coeffs,
                                                             double* __restrict__ epart) {
  __shared__ double red[kVqeBlock / kWave];
  const unsigned long long N = 1ull << n;
  const double2* __restrict__ p = phi0 + (size_t)blockIdx.y * N;
  double2* __restrict__ l = lam0 + (size_t)blockIdx.y * N;
  const double* cb = coeffs ? coeffs + (size_t)blockIdx.y * nterms : nullptr;
  double e = 0.0;
  for (unsigned long long j = (unsigned long long)blockIdx.x * kVqeBlock + threadIdx.x; j < N;
       j += (unsigned long long)gridDim.x * kVqeBlock) {
    vd2 acc = FIRST ? mk(0.0, 0.0) : ld(l + j);
    for (int i = 0; i < cnt; ++i) {
      const int t = tidx[i];
      const VqeTerm T = terms[t];
      const double tc = cb ? cb[t] : T.c;
      const unsigned long long k = j ^ T.x;
      vd2 v = ld(p + k);
      switch (T.y & 3) {
        case 1: v = mk(-v.y, v.x); break;
        case 2: v = mk(-v.x, -v.y); break;
        case 3: v = mk(v.y, -v.x); break;
        default: break;
      }
      const double c = (__popcll(k & T.z) & 1) ? -tc : tc;
      acc.x = fma(c, v.x, acc.x);
      acc.y = fma(c, v.y, acc.y);
    }
    st(l + j, acc);
    if (LAST) {
      const vd2 v = ld(p + j);
      e += v.x * acc.x + v.y * acc.y;
    }
  }
  if (LAST) {
    e = wave_sum(e);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < kVqeBlock / kWave; ++w) s += red[w];
      epart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
  }
}

// Backward step over all states; gradient partials gpart[(b * nslots + slot) * G + block]
__global__ __launch_bounds__(kVqeBlock) void k_vqe_adjoint(double2* __restrict__ phi, double2* __restrict__ lam,
                                                           int n, VqeOp op, const double2* __restrict__ fixed,
                                                           const double* __restrict__ theta, int P, int nslots,
                                                           double* __restrict__ gpart) {
  __shared__ double red[kVqeBlock / kWave];
  const unsigned long long N = 1ull << n;
  double2* pv = phi + (size_t)blockIdx.y * N;
  double2* lv = lam + (size_t)blockIdx.y * N;
  const double* th = theta + (size_t)blockIdx.y * P;
  const unsigned long long tid = (unsigned long long)blockIdx.x * kVqeBlock + threadIdx.x;
  const unsigned long long nt = (unsigned long long)gridDim.x * kVqeBlock;
  double g = 0.0;
  if (op.kind == OP_ROT) {
    const M2 m = rot_matrix(op.axis, th[op.param], true);
    const unsigned long long off = 1ull << op.q0, np = N >> 1;
    unsigned long long p = tid;
    // kU pairs per step; the gradient terms are added in pair order
    for (; p + (kU - 1) * nt < np; p += kU * nt) {
      unsigned long long i0[kU];
      vd2 p0[kU], p1[kU], l0[kU], l1[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        i0[u] = ins0l(p + u * nt, op.q0);
        p0[u] = ld(pv + i0[u]);
        p1[u] = ld(pv + i0[u] + off);
        l0[u] = ld(lv + i0[u]);
        l1[u] = ld(lv + i0[u] + off);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        g += pair_grad(op.axis, p0[u], p1[u], l0[u], l1[u]);
        st(pv + i0[u], cfma(m.m0, p0[u], cmul(m.m1, p1[u])));
        st(pv + i0[u] + off, cfma(m.m2, p0[u], cmul(m.m3, p1[u])));
        st(lv + i0[u], cfma(m.m0, l0[u], cmul(m.m1, l1[u])));
        st(lv + i0[u] + off, cfma(m.m2, l0[u], cmul(m.m3, l1[u])));
      }
    }
    for (; p < np; p += nt) {
      const unsigned long long i0 = ins0l(p, op.q0);
      const vd2 p0 = ld(pv + i0), p1 = ld(pv + i0 + off);
      const vd2 l0 = ld(lv + i0), l1 = ld(lv + i0 + off);
      g += pair_grad(op.axis, p0, p1, l0, l1);
      st(pv + i0, cfma(m.m0, p0, cmul(m.m1, p1)));
      st(pv + i0 + off, cfma(m.m2, p0, cmul(m.m3, p1)));
      st(lv + i0, cfma(m.m0, l0, cmul(m.m1, l1)));
      st(lv + i0 + off, cfma(m.m2, l0, cmul(m.m3, l1)));
    }
  } else {   // OP_RZZ
    vd2 e, o;
    rzz_phases(th[op.param], true, e, o);
    unsigned long long j = tid;
    for (; j + (kU - 1) * nt < N; j += kU * nt) {
      vd2 x[kU], y[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        x[u] = ld(pv + j + u * nt);
        y[u] = ld(lv + j + u * nt);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const unsigned long long i = j + u * nt;
        const unsigned par = (unsigned)(((i >> op.q0) ^ (i >> op.q1)) & 1ull);
        const double t = y[u].x * x[u].y - y[u].y * x[u].x;
        g += par ? -t : t;
        st(pv + i, cmul(par ? o : e, x[u]));
        st(lv + i, cmul(par ? o : e, y[u]));
      }
    }
    for (; j < N; j += nt) {
      const unsigned par = (unsigned)(((j >> op.q0) ^ (j >> op.q1)) & 1ull);
      const vd2 p = ld(pv + j), l = ld(lv + j);
      const double t = l.x * p.y - l.y * p.x;
      g += par ? -t : t;
      st(pv + j, cmul(par ? o : e, p));
      st(lv + j, cmul(par ? o : e, l));
    }
  }
  g = wave_sum(g);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = g;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kVqeBlock / kWave; ++w) s += red[w];
    gpart[((size_t)blockIdx.y * nslots + op.slot) * gridDim.x + blockIdx.x] = s;
  }
}

// Closing reductions in a fixed order that depends only on G: each slot's G
// gradient partials are summed by one wave (lanes stride over the partials,
// then a fixed shuffle tree) into ssum; then one workgroup per state sums
// the energy partials the same way and each parameter adds its slots in slot
// order.
constexpr int kFinBlock = 256;

// Slot sums: workgroup (chunk, b) gives one slot to each wave.
__global__ __launch_bounds__(kFinBlock) void k_vqe_slot_sums(const double* __restrict__ gpart, int G, int nslots,
                                                             double* __restrict__ ssum) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & (kWave - 1);
  const int s = blockIdx.x * (kFinBlock / kWave) + threadIdx.x / kWave;
  if (s >= nslots) return;
  const double* gp = gpart + ((size_t)b * nslots + s) * G;
  double v = 0.0;
  for (int k = lane; k < G; k += kWave) v += gp[k];
  v = wave_sum(v);
  if (lane == 0) ssum[(size_t)b * nslots + s] = v;
}

__global__ __launch_bounds__(kFinBlock) void k_vqe_finish(const double* __restrict__ epart, int G, int nslots,
                                                          const int* __restrict__ slot_param, int P,
                                                          const double* __restrict__ ssum, double* __restrict__ E,
                                                          double* __restrict__ grad) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (wave == 0) {
    double e = 0.0;
    for (int k = lane; k < G; k += kWave) e += epart[(size_t)b * G + k];
    e = wave_sum(e);
    if (lane == 0) E[b] = e;
  }
  if (!grad) return;
  for (int p = threadIdx.x; p < P; p += kFinBlock) {
    double g = 0.0;
    for (int s = 0; s < nslots; ++s)
      if (slot_param[s] == p) g += ssum[(size_t)b * nslots + s];
    grad[(size_t)b * P + p] = g;
  }
}

}  // namespace

namespace {
// ---------------------------------------------------------------------------
// Fused path (any n > tile): gates grouped into k-qubit blocks as for state
// vectors; the forward pass runs the register-blocked fused kernel over all
// B states with a per-vector matrix table, the backward pass holds tiles of
// phi and lambda in LDS and sweeps each block's gates in reverse.
// ---------------------------------------------------------------------------
struct VqeBwdOp {
  int kind;    // 0 rotation, 1 RZZ, 2 fixed 2x2, 3 CX, 4 CZ, 5 SWAP
  int lo, hi;  // sorted tile-local bits
  int b0, b1;  // tile-local bits in operator order
  int axis;    // rotation axis
  int slot;    // gradient slot or -1
  int mat;     // index of the adjoint matrix in the per-vector table (double2 units)
};

constexpr int kBwdBlock = 256;
constexpr int kBwdMaxOps = 128;
constexpr int kBwdStage = 8;   // tile entries per thread staged together (loads issued before LDS writes)

__device__ __forceinline__ unsigned long long bwd_index(unsigned long long base, unsigned l, unsigned cmask, int c,
                                                        int m, const FusedBlockDev& blk) {
  unsigned long long g = base | (l & cmask);
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < m && ((l >> (c + i)) & 1u)) g |= 1ull << blk.hi[i];
  return g;
}

// Per-vector matrix table: for op i, entries [8i, 8i+4) hold the forward
// matrix (2x2 row-major, or the 4 diagonal entries of RZZ / CZ indexed by
// u = bit q0 + 2 bit q1) and [8i+4, 8i+8) the adjoint.  Every case stores
// inside its own branch.
__global__ __launch_bounds__(256) void k_vqe_mats(const VqeOp* __restrict__ ops, int nops,
                                                  const double2* __restrict__ fixed,
                                                  const double* __restrict__ theta, int P,
                                                  double2* __restrict__ table) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nops) return;
  const int b = blockIdx.y;
  const VqeOp op = ops[i];
  const double* th = theta + (size_t)b * P;
  double2* t = table + ((size_t)b * nops + i) * 8;
  if (op.kind == OP_ROT) {
    const M2 f = rot_matrix(op.axis, th[op.param], false);
    st(t + 0, f.m0); st(t + 1, f.m1); st(t + 2, f.m2); st(t + 3, f.m3);
    const M2 a = rot_matrix(op.axis, th[op.param], true);
    st(t + 4, a.m0); st(t + 5, a.m1); st(t + 6, a.m2); st(t + 7, a.m3);
  } else if (op.kind == OP_RZZ) {
    vd2 e, o;
    rzz_phases(th[op.param], false, e, o);
    st(t + 0, e); st(t + 1, o); st(t + 2, o); st(t + 3, e);
    rzz_phases(th[op.param], true, e, o);
    st(t + 4, e); st(t + 5, o); st(t + 6, o); st(t + 7, e);
  } else if (op.kind == OP_FIX1) {
    for (int k = 0; k < 8; ++k) t[k] = fixed[8 * op.mat + k];
  } else if (op.kind == OP_CZ) {
    for (int k = 0; k < 8; ++k) st(t + k, mk((k & 3) == 3 ? -1.0 : 1.0, 0.0));
  } else {
    for (int k = 0; k < 8; ++k) st(t + k, mk(0.0, 0.0));
  }
}

__global__ __launch_bounds__(kBwdBlock) void k_vqe_bwd_tile(double2* __restrict__ phi0, double2* __restrict__ lam0,
                                                            int n, FusedBlockDev blk,
                                                            const VqeBwdOp* __restrict__ ops,
                                                            const double2* __restrict__ table0, int mat_stride,
                                                            int nslots, double* __restrict__ gpart,
                                                            unsigned long long ntiles) {
  extern __shared__ double2 sh[];
  __shared__ double acc[kBwdMaxOps][kBwdBlock / kWave];
  constexpr int NW = kBwdBlock / kWave;
  const int c = blk.c, m = blk.m, k = c + m;
  const unsigned len = 1u << k;
  double2* tp = sh;
  double2* tl = sh + len;
  const unsigned long long N = 1ull << n;
  double2* __restrict__ phi = phi0 + (size_t)blockIdx.y * N;
  double2* __restrict__ lam = lam0 + (size_t)blockIdx.y * N;
  const double2* __restrict__ table = table0 + (size_t)blockIdx.y * mat_stride;
  
  const unsigned cmask = (1u << c) - 1u;
  const unsigned tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  for (int i = tid; i < blk.op_count * NW; i += kBwdBlock) acc[i / NW][i % NW] = 0.0;
  for (unsigned long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    unsigned long long base = tile << c;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < m) {
        const int q = blk.hi[i];
        base = ((base >> q) << (q + 1)) | (base & ((1ull << q) - 1ull));
      }
    }
    __syncthreads();
    if (len >= kBwdStage * kBwdBlock) {
      for (unsigned l0 = tid; l0 < len; l0 += kBwdStage * kBwdBlock) {
        vd2 rp[kBwdStage], rl[kBwdStage];
#pragma unroll
        for (int j = 0; j < kBwdStage; ++j) {
          const unsigned long long g = bwd_index(base, l0 + j * kBwdBlock, cmask, c, m, blk);
          rp[j] = ld(phi + g);
          rl[j] = ld(lam + g);
        }
#pragma unroll
        for (int j = 0; j < kBwdStage; ++j) {
          st(tp + l0 + j * kBwdBlock, rp[j]);
          st(tl + l0 + j * kBwdBlock, rl[j]);
        }
      }
    } else {
      for (unsigned l = tid; l < len; l += kBwdBlock) {
        const unsigned long long g = bwd_index(base, l, cmask, c, m, blk);
        tp[l] = phi[g];
        tl[l] = lam[g];
      }
    }
    for (int oi = 0; oi < blk.op_count; ++oi) {
      const VqeBwdOp op = ops[blk.op_begin + oi];
      const double2* M = table + op.mat;
      __syncthreads();
      double g = 0.0;
      if (op.kind == 0 || op.kind == 2) {
        const vd2 m0 = ld(M), m1 = ld(M + 1), m2 = ld(M + 2), m3 = ld(M + 3);
        const unsigned off = 1u << op.lo;
        for (unsigned p = tid; p < (len >> 1); p += kBwdBlock) {
          const unsigned i0 = ins0(p, op.lo);
          const vd2 p0 = ld(tp + i0), p1 = ld(tp + i0 + off);
          const vd2 l0 = ld(tl + i0), l1 = ld(tl + i0 + off);
          if (op.kind == 0) g += pair_grad(op.axis, p0, p1, l0, l1);
          st(tp + i0, cfma(m0, p0, cmul(m1, p1)));
          st(tp + i0 + off, cfma(m2, p0, cmul(m3, p1)));
          st(tl + i0, cfma(m0, l0, cmul(m1, l1)));
          st(tl + i0 + off, cfma(m2, l0, cmul(m3, l1)));
        }
      } else if (op.kind == 1 || op.kind == 4) {
        const vd2 d0 = ld(M), d1 = ld(M + 1), d2 = ld(M + 2), d3 = ld(M + 3);
        for (unsigned l = tid; l < len; l += kBwdBlock) {
          const bool a = (l >> op.b0) & 1u, b = (l >> op.b1) & 1u;
          const vd2 f = b ? (a ? d3 : d2) : (a ? d1 : d0);
          const vd2 pv = ld(tp + l), lv = ld(tl + l);
          if (op.kind == 1) {
            const double t = lv.x * pv.y - lv.y * pv.x;   // Im(conj(l) p) times the ZZ eigenvalue
            g += (a != b) ? -t : t;
          }
          st(tp + l, cmul(f, pv));
          st(tl + l, cmul(f, lv));
        }
      } else {   // 3 CX (control b0, target b1), 5 SWAP
        const unsigned oa = 1u << op.b0;
        const unsigned ob = op.kind == 3 ? (1u << op.b0) + (1u << op.b1) : (1u << op.b1);
        for (unsigned p = tid; p < (len >> 2); p += kBwdBlock) {
          const unsigned b = ins0(ins0(p, op.lo), op.hi);
          const vd2 x = ld(tp + b + oa), y = ld(tp + b + ob);
          st(tp + b + oa, y);
          st(tp + b + ob, x);
          const vd2 u = ld(tl + b + oa), w = ld(tl + b + ob);
          st(tl + b + oa, w);
          st(tl + b + ob, u);
        }
      }
      if (op.slot >= 0) {
        const double w = wave_sum(g);
        if (lane == 0) acc[oi][wave] += w;
      }
    }
    __syncthreads();
    if (len >= kBwdStage * kBwdBlock) {
      for (unsigned l0 = tid; l0 < len; l0 += kBwdStage * kBwdBlock) {
        vd2 rp[kBwdStage], rl[kBwdStage];
#pragma unroll
        for (int j = 0; j < kBwdStage; ++j) {
          rp[j] = ld(tp + l0 + j * kBwdBlock);
          rl[j] = ld(tl + l0 + j * kBwdBlock);
        }
#pragma unroll
        for (int j = 0; j < kBwdStage; ++j) {
          const unsigned long long g = bwd_index(base, l0 + j * kBwdBlock, cmask, c, m, blk);
          st(phi + g, rp[j]);
          st(lam + g, rl[j]);
        }
      }
    } else {
      for (unsigned l = tid; l < len; l += kBwdBlock) {
        const unsigned long long g = bwd_index(base, l, cmask, c, m, blk);
        phi[g] = tp[l];
        lam[g] = tl[l];
      }
    }
  }
  __syncthreads();
  for (int oi = tid; oi < blk.op_count; oi += kBwdBlock) {
    const int slot = ops[blk.op_begin + oi].slot;
    if (slot < 0) continue;
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += acc[oi][w];
    gpart[((size_t)blockIdx.y * nslots + slot) * gridDim.x + blockIdx.x] = v;
  }
}

// ---------------------------------------------------------------------------
// Register-blocked backward sweep.  The block's reversed gates are split into
// phases over R register bits (as in the forward kernel); per phase each
// thread holds the 2^R amplitudes of phi and of lambda that differ on those
// bits and un-applies the phase's gates in registers, accumulating each
// parametrised gate's Im<lambda|P|phi> before un-applying it.  Tiles of phi
// and lambda are exchanged through LDS between phases.
// ---------------------------------------------------------------------------
struct VqeBwdRop {
  int kind;    // 0 rotation, 1 RZZ, 2 fixed 2x2, 3 CX, 4 CZ, 5 SWAP
  int r0, r1;  // register-bit indices in operator order (r1 for 2-qubit ops)
  int axis;    // rotation axis
  int slot;    // gradient slot or -1
  int mat;     // index of the adjoint matrix in the per-vector table (double2 units)
  int code;    // switch index: 4 v + r0 for 2x2 ops (v = axis, 3 = fixed);
               // 16 + 16 w + 4 r0 + r1 for 2q ops (w: 0 RZZ, 1 CZ, 2 CX, 3 SWAP)
  int pad1;
};
inline int bwd_rop_code(const VqeBwdRop& o) {
  if (o.kind == 0 || o.kind == 2) return 4 * (o.kind == 2 ? 3 : o.axis) + o.r0;
  const int w = o.kind == 1 ? 0 : o.kind == 4 ? 1 : o.kind == 3 ? 2 : 3;
  return 16 + 16 * w + 4 * o.r0 + o.r1;
}

constexpr int kBwdRbMaxWaves = 4;   // tiles of at most 2^11 entries at 3 register bits
constexpr int kBwdMaxTileBits = 11;

__device__ __forceinline__ unsigned padl_b(unsigned l) { return l + (l >> 4); }
// one padded tile of 2^k entries (one extra entry per 16)
inline size_t bwd_rb_tile_bytes(int k) { return sizeof(double2) * ((1u << k) + (1u << k) / 16); }

// Im(conj(a) b)
__device__ __forceinline__ double imcb(vd2 a, vd2 b) { return a.x * b.y - a.y * b.x; }
// Re(conj(a) b)
__device__ __forceinline__ double recb(vd2 a, vd2 b) { return a.x * b.x + a.y * b.y; }

// Rotation about axis AX (0 X, 1 Y, 2 Z; -1: fixed gate, no gradient) on
// register bit B: the generator's term Im<l|P|p> of the pair (as in
// pair_grad, one axis only), then the adjoint 2x2 on both vectors; RZ's
// adjoint is diagonal (M[0], M[3]).
template <int NV, int B, int AX>
__device__ __forceinline__ void bw_rot(vd2 (&p)[NV], vd2 (&l)[NV], const double2* __restrict__ M, double& g) {
  const vd2 m0 = ld(M), m1 = ld(M + 1), m2 = ld(M + 2), m3 = ld(M + 3);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const vd2 p0 = p[j], p1 = p[k], l0 = l[j], l1 = l[k];
    if constexpr (AX == 0) g += imcb(l0, p1) + imcb(l1, p0);
    if constexpr (AX == 1) g += recb(l1, p0) - recb(l0, p1);
    if constexpr (AX == 2) g += imcb(l0, p0) - imcb(l1, p1);
    if constexpr (AX == 2) {
      p[j] = cmul(m0, p0);
      p[k] = cmul(m3, p1);
      l[j] = cmul(m0, l0);
      l[k] = cmul(m3, l1);
    } else if constexpr (AX == 1) {
      // RY adjoint: a real 2x2 (the zero imaginary parts are not multiplied;
      // the rounding is that of the complex form)
      p[j] = mk(fma(m0.x, p0.x, m1.x * p1.x), fma(m0.x, p0.y, m1.x * p1.y));
      p[k] = mk(fma(m2.x, p0.x, m3.x * p1.x), fma(m2.x, p0.y, m3.x * p1.y));
      l[j] = mk(fma(m0.x, l0.x, m1.x * l1.x), fma(m0.x, l0.y, m1.x * l1.y));
      l[k] = mk(fma(m2.x, l0.x, m3.x * l1.x), fma(m2.x, l0.y, m3.x * l1.y));
    } else if constexpr (AX == 0) {
      // RX adjoint: real diagonal, imaginary off-diagonal entries
      p[j] = mk(fma(m0.x, p0.x, -(m1.y * p1.y)), fma(m0.x, p0.y, m1.y * p1.x));
      p[k] = mk(fma(-m2.y, p0.y, m3.x * p1.x), fma(m2.y, p0.x, m3.x * p1.y));
      l[j] = mk(fma(m0.x, l0.x, -(m1.y * l1.y)), fma(m0.x, l0.y, m1.y * l1.x));
      l[k] = mk(fma(-m2.y, l0.y, m3.x * l1.x), fma(m2.y, l0.x, m3.x * l1.y));
    } else {
      p[j] = cfma(m0, p0, cmul(m1, p1));
      p[k] = cfma(m2, p0, cmul(m3, p1));
      l[j] = cfma(m0, l0, cmul(m1, l1));
      l[k] = cfma(m2, l0, cmul(m3, l1));
    }
  }
}

// Diagonal 2-qubit op on register bits B0 (u bit 0), B1 (u bit 1); with grad,
// the ZZ generator's term Im(conj(l) p) times its eigenvalue.
template <int NV, int B0, int B1>
__device__ __forceinline__ void bw_diag2(vd2 (&p)[NV], vd2 (&l)[NV], const double2* __restrict__ M, bool grad,
                                         double& g) {
  const vd2 d[4] = {ld(M), ld(M + 1), ld(M + 2), ld(M + 3)};
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int a = (j >> B0) & 1, b = (j >> B1) & 1;
    if (grad) {
      const double t = l[j].x * p[j].y - l[j].y * p[j].x;
      g += (a != b) ? -t : t;
    }
    p[j] = cmul(d[a + 2 * b], p[j]);
    l[j] = cmul(d[a + 2 * b], l[j]);
  }
}

template <int NV, int B0, int B1, int OA, int OB>
__device__ __forceinline__ void bw_swap(vd2 (&p)[NV], vd2 (&l)[NV]) {
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (j & ((1 << B0) | (1 << B1))) continue;
    vd2 t = p[j | OA];
    p[j | OA] = p[j | OB];
    p[j | OB] = t;
    t = l[j | OA];
    l[j | OA] = l[j | OB];
    l[j | OB] = t;
  }
}

template <int R, int B, int AX>
__device__ __forceinline__ void bw_c1(vd2 (&p)[1 << R], vd2 (&l)[1 << R], const double2* M, double& g) {
  if constexpr (B < R) bw_rot<(1 << R), B, AX>(p, l, M, g);
}
template <int R, int B0, int B1, int W>
__device__ __forceinline__ void bw_c2(vd2 (&p)[1 << R], vd2 (&l)[1 << R], const double2* M, double& g) {
  constexpr int NV = 1 << R;
  if constexpr (B0 < R && B1 < R) {
    if constexpr (W == 0) bw_diag2<NV, B0, B1>(p, l, M, true, g);                             // RZZ
    else if constexpr (W == 1) bw_diag2<NV, B0, B1>(p, l, M, false, g);                       // CZ
    else if constexpr (W == 2) bw_swap<NV, B0, B1, (1 << B0), (1 << B0) | (1 << B1)>(p, l);  // CX: control B0
    else bw_swap<NV, B0, B1, (1 << B0), (1 << B1)>(p, l);                                    // SWAP
  }
}

// One adjoint gate: a single switch over its code (bwd_rop_code).
template <int R>
__device__ __forceinline__ void bw_apply(int code, vd2 (&p)[1 << R], vd2 (&l)[1 << R], const double2* __restrict__ M,
                                         double& g) {
#define NWQ_BW1(V, AX) \
  case 4 * V + 0: bw_c1<R, 0, AX>(p, l, M, g); break; \
  case 4 * V + 1: bw_c1<R, 1, AX>(p, l, M, g); break; \
  case 4 * V + 2: bw_c1<R, 2, AX>(p, l, M, g); break; \
  case 4 * V + 3: bw_c1<R, 3, AX>(p, l, M, g); break;
#define NWQ_BW2(W) \
  case 16 + 16 * W + 1: bw_c2<R, 0, 1, W>(p, l, M, g); break; \
  case 16 + 16 * W + 2: bw_c2<R, 0, 2, W>(p, l, M, g); break; \
  case 16 + 16 * W + 3: bw_c2<R, 0, 3, W>(p, l, M, g); break; \
  case 16 + 16 * W + 4: bw_c2<R, 1, 0, W>(p, l, M, g); break; \
  case 16 + 16 * W + 6: bw_c2<R, 1, 2, W>(p, l, M, g); break; \
  case 16 + 16 * W + 7: bw_c2<R, 1, 3, W>(p, l, M, g); break; \
  case 16 + 16 * W + 8: bw_c2<R, 2, 0, W>(p, l, M, g); break; \
  case 16 + 16 * W + 9: bw_c2<R, 2, 1, W>(p, l, M, g); break; \
  case 16 + 16 * W + 11: bw_c2<R, 2, 3, W>(p, l, M, g); break; \
  case 16 + 16 * W + 12: bw_c2<R, 3, 0, W>(p, l, M, g); break; \
  case 16 + 16 * W + 13: bw_c2<R, 3, 1, W>(p, l, M, g); break; \
  case 16 + 16 * W + 14: bw_c2<R, 3, 2, W>(p, l, M, g); break;
  switch (code) {
    NWQ_BW1(0, 0)
    NWQ_BW1(1, 1)
    NWQ_BW1(2, 2)
    NWQ_BW1(3, -1)
    NWQ_BW2(0)
    NWQ_BW2(1)
    NWQ_BW2(2)
    NWQ_BW2(3)
    default: break;
  }
#undef NWQ_BW1
#undef NWQ_BW2
}

// Global loads and stores of tile entries; NT: non-temporal (each entry of
// phi and lambda is read and written once per block).
template <bool NT>
__device__ __forceinline__ vd2 bgld(const double2* p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const vd2*>(p));
  else return ld(p);
}
template <bool NT>
__device__ __forceinline__ void bgst(double2* p, vd2 v) {
  if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<vd2*>(p));
  else st(p, v);
}

template <int R, bool NT>
__global__ __launch_bounds__(kWave * kBwdRbMaxWaves) void k_vqe_bwd_rb(double2* __restrict__ phi0,
                                                                      double2* __restrict__ lam0, int n,
                                                                      FusedBlockDev blk,
                                                                      const FusedPhase* __restrict__ phases,
                                                                      const VqeBwdRop* __restrict__ ops,
                                                                      const double2* __restrict__ table0,
                                                                      int mat_stride, int nslots,
                                                                      double* __restrict__ gpart,
                                                                      unsigned long long ntiles) {
  constexpr int NV = 1 << R;
  extern __shared__ double2 sh[];
  __shared__ double acc[kBwdMaxOps][kBwdRbMaxWaves];
  const int c = blk.c, m = blk.m, k = c + m;
  const unsigned len = 1u << k;
  const unsigned nt = len >> R;
  double2* tp = sh;
  double2* tl = sh + padl_b(len);
  const unsigned long long N = 1ull << n;
  double2* __restrict__ phi = phi0 + (size_t)blockIdx.y * N;
  double2* __restrict__ lam = lam0 + (size_t)blockIdx.y * N;
  const double2* __restrict__ table = table0 + (size_t)blockIdx.y * mat_stride;
  
  const unsigned cmask = (1u << c) - 1u;
  const unsigned tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int NW = (int)(nt + kWave - 1) / kWave;
  const int op0 = phases[blk.op_begin].op_begin;
  const FusedPhase last = phases[blk.op_begin + blk.op_count - 1];
  const int nops = last.op_begin + last.op_count - op0;
  for (int i = tid; i < nops * kBwdRbMaxWaves; i += nt) acc[i / kBwdRbMaxWaves][i % kBwdRbMaxWaves] = 0.0;
  const unsigned long long glane = bwd_index(0ull, tid, cmask, c, m, blk);
  auto tile_off = [&](unsigned long long tile) {
    unsigned long long base = tile << c;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < m) {
        const int q = blk.hi[i];
        base = ((base >> q) << (q + 1)) | (base & ((1ull << q) - 1ull));
      }
    }
    return base + glane;
  };
  // The tile's entries of phi and lambda are loaded one tile ahead: the
  // loads of the next tile are in flight while this one runs its phases
  // (tiles are disjoint, so the early read is safe).  A tile's results leave
  // LDS at the end of its trip and go to HBM after the next tile is staged,
  // ahead of the next loads: the vector memory counter retires in issue
  // order, so stores issued after those loads would make the next trip's
  // wait for them cover the stores' completion too.
  vd2 fp[NV], fl[NV], rp[NV], rl[NV];
  unsigned long long prev = ~0ull;
  if (blockIdx.x < ntiles) {
    const unsigned long long o = tile_off(blockIdx.x);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      fp[j] = bgld<NT>(phi + o + blk.joff[j]);
      fl[j] = bgld<NT>(lam + o + blk.joff[j]);
    }
  }
  for (unsigned long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    {
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        st(tp + padl_b(tid + j * nt), fp[j]);
        st(tl + padl_b(tid + j * nt), fl[j]);
      }
      if (prev != ~0ull) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          bgst<NT>(phi + prev + blk.joff[j], rp[j]);
          bgst<NT>(lam + prev + blk.joff[j], rl[j]);
        }
      }
      const unsigned long long nx = tile + gridDim.x;
      if (nx < ntiles) {
        const unsigned long long o = tile_off(nx);
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          fp[j] = bgld<NT>(phi + o + blk.joff[j]);
          fl[j] = bgld<NT>(lam + o + blk.joff[j]);
        }
      }
    }
    for (int pi = 0; pi < blk.op_count; ++pi) {
      const FusedPhase ph = phases[blk.op_begin + pi];
      unsigned dep = tid;
#pragma unroll
      for (int r = 0; r < R; ++r) dep = ((dep >> ph.reg[r]) << (ph.reg[r] + 1)) | (dep & ((1u << ph.reg[r]) - 1u));
      double2* __restrict__ sp = tp + padl_b(dep);
      double2* __restrict__ sl = tl + padl_b(dep);
      __syncthreads();
      vd2 vp[NV], vl[NV];
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        vp[j] = ld(sp + ph.ld_off[j]);
        vl[j] = ld(sl + ph.ld_off[j]);
      }
      for (int oi = 0; oi < ph.op_count; ++oi) {
        const VqeBwdRop op = ops[ph.op_begin + oi];
        double g = 0.0;
        bw_apply<R>(op.code, vp, vl, table + op.mat, g);
        if (op.slot >= 0) {
          const double w = wave_sum_full(g);   // tiles of >= 2^9 entries: whole waves
          if (lane == 0) acc[ph.op_begin + oi - op0][wave] += w;
        }
      }
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        st(sp + ph.st_off[j], vp[j]);
        st(sl + ph.st_off[j], vl[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      rp[j] = ld(tp + padl_b(tid + j * nt));
      rl[j] = ld(tl + padl_b(tid + j * nt));
    }
    prev = tile_off(tile);
  }
  if (prev != ~0ull) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      bgst<NT>(phi + prev + blk.joff[j], rp[j]);
      bgst<NT>(lam + prev + blk.joff[j], rl[j]);
    }
  }
  __syncthreads();
  for (int oi = tid; oi < nops; oi += nt) {
    const int slot = ops[op0 + oi].slot;
    if (slot < 0) continue;
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += acc[oi][w];
    gpart[((size_t)blockIdx.y * nslots + slot) * gridDim.x + blockIdx.x] = v;
  }
}

}  // namespace

// ===========================================================================
// Host: context
// ===========================================================================
struct VqeConfig {
  int mode = 0;        // 0 auto, 1 LDS-resident, 2 global per-gate (graph)
  int threads = 256;   // LDS kernel block size
  int blocks_per_state = 0;   // global path: 0 = derived from n
};

}  // namespace nwq

struct nwq_vqe {
  int n = 0, P = 0, nops = 0, nterms = 0, nslots = 0;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;       // own stream (graph capture needs a non-null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<nwq::VqeOp> ops;
  std::vector<int> slot_param;
  nwq::VqeOp* d_ops = nullptr;
  double2* d_fixed = nullptr;
  nwq::VqeTerm* d_terms = nullptr;
  std::vector<nwq::VqeTerm> terms;   // host copy of the term table
  int* d_slot_param = nullptr;
  // global path buffers
  int Bcap = 0;
  double2* d_phi = nullptr;
  double2* d_lam = nullptr;
  double* d_epart = nullptr;
  double* d_gpart = nullptr;
  double* d_theta = nullptr;   // staging copies for graph replays
  double* d_E = nullptr;
  double* d_grad = nullptr;
  double* d_coeffs = nullptr;  // staging copy of per-vector coefficients
  double2* d_table = nullptr;  // fused path: per-vector matrix table [B][nops][8]
  double* d_ssum = nullptr;    // per-slot gradient sums [B][nslots]
  // fused path program (built on first use)
  bool fused_built = false;
  int fused_k = 12;
  int low_bits = 0;            // low tile bits of the planned blocks: 0 = kVqeLowBits
  int fused_rbits = 4;         // register bits per phase of the forward kernel
  bool bwd_rb = false;         // backward sweep register-blocked (3 bits) when every tile has >= 2^9 entries
  size_t fused_rop_off = 0;    // offset of the register-blocked backward ops in d_fused
  std::vector<nwq::FusedBlockDev> fwd_blocks, bwd_blocks;
  // backward dispatches of the first planned block (the last of the sweep):
  // phi is non-zero in tile 0 only there (it equals that block applied to
  // |0...0>), and lambda is not read after the sweep, so they run tile 0 only
  std::vector<char> bwd_tile0;
  // lambda = H phi of the fused schedule: tiled passes (and a gather pass for
  // terms that fit no tile), in launch order
  struct HLaunch {
    int wide;            // 1: k_vqe_hphi_wide over the term indices at widx[w_begin .. w_begin + w_count)
    nwq::HPass p;        // tiled pass (p.t_begin indexes the HTerm table)
    int w_begin, w_count;
  };
  std::vector<HLaunch> hlaunch;
  size_t fused_hterm_off = 0, fused_widx_off = 0;
  void* d_fused = nullptr;     // [forward phases][forward ops][backward ops]
  size_t fused_ops_off = 0, fused_bwd_off = 0;
  nwq::VqeConfig cfg;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;   // (B, want_grad) -> exec
  int fused_flags = 3;         // fused schedule: bit 0 non-temporal tile loads and stores, bit 1 direct
                               // HBM loads / stores of a forward block's first / last phase
  size_t program_bytes = 0;    // device bytes of d_ops, d_fixed, d_terms, d_slot_param
  size_t fused_bytes = 0;      // device bytes of d_fused once built
};

namespace nwq {

static int vqe_fail(int code, const std::string& m) { return set_error(code, m); }

// Workgroups per state of the per-gate and fused schedules.  The partial
// sums (and so the rounding) depend on it, so it is fixed per context and
// never derived from B; the default fills the chip with one state (up to
// 1024 workgroups of 4 pairs per thread), the batch adds the rest.
static int blocks_per_state(const nwq_vqe* h) {
  if (h->cfg.blocks_per_state > 0) return h->cfg.blocks_per_state;
  const unsigned long long pairs = 1ull << (h->n - 1);
  const unsigned long long b = (pairs + kVqeBlock * 4 - 1) / (kVqeBlock * 4);
  return (int)std::max<unsigned long long>(1, std::min<unsigned long long>(b, 1024));
}

static size_t lds_bytes(const nwq_vqe* h, int threads, bool want_grad) {
  const size_t N = 1ull << h->n;
  const int NW = threads / kWave;
  return (want_grad ? 2 : 1) * N * sizeof(double2) + (size_t)NW * sizeof(double) +
         (want_grad ? (size_t)h->nslots * NW * sizeof(double) : 0);
}

static bool lds_fits(const nwq_vqe* h, int threads, bool want_grad) {
  return h->n <= 12 && lds_bytes(h, threads, want_grad) <= 160 * 1024;
}

static int launch_lds(nwq_vqe* h, int B, const double* theta, const double* coeffs, double* E, double* grad,
                      hipStream_t s) {
  const int T = h->cfg.threads;
  const size_t lds = lds_bytes(h, T, grad != nullptr);
  const int grid = std::min(B, 4096);
#define NWQ_VQE_LDS(NTV)                                                                                     \
  do {                                                                                                       \
    if (lds > 65536) (void)enable_dynamic_lds((const void*)k_vqe_lds<NTV>);                                  \
    hipLaunchKernelGGL(k_vqe_lds<NTV>, dim3(grid), dim3(NTV), lds, s, h->n, h->d_ops, h->nops, h->d_fixed,   \
                       h->d_terms, h->nterms, h->nslots, h->d_slot_param, theta, h->P, B, coeffs, E, grad);  \
  } while (0)
  switch (T) {
    case 64: NWQ_VQE_LDS(64); break;
    case 128: NWQ_VQE_LDS(128); break;
    case 512: NWQ_VQE_LDS(512); break;
    case 1024: NWQ_VQE_LDS(1024); break;
    default: NWQ_VQE_LDS(256); break;
  }
#undef NWQ_VQE_LDS
  return check_hip(hipGetLastError(), "k_vqe_lds");
}

// Device bytes of the global-path buffers per parameter vector (what
// ensure_global allocates for each unit of its capacity).
static size_t global_bytes_per_vector(const nwq_vqe* h) {
  const size_t N = 1ull << h->n;
  const size_t G = (size_t)blocks_per_state(h);
  const size_t P = std::max(1, h->P), S = std::max(1, h->nslots), T = std::max(1, h->nterms), O = std::max(1, h->nops);
  return 2 * N * sizeof(double2) + G * sizeof(double) + S * G * sizeof(double) + 2 * P * sizeof(double) +
         sizeof(double) + T * sizeof(double) + O * 8 * sizeof(double2) + S * sizeof(double);
}

static int ensure_global(nwq_vqe* h, int B) {
  if (B <= h->Bcap) return NWQ_OK;
  int rc = check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  h->graphs.clear();
  for (void* p : {(void*)h->d_phi, (void*)h->d_lam, (void*)h->d_epart, (void*)h->d_gpart, (void*)h->d_theta,
                  (void*)h->d_E, (void*)h->d_grad, (void*)h->d_coeffs, (void*)h->d_table, (void*)h->d_ssum})
    if (p) (void)hipFree(p);
  h->d_phi = h->d_lam = h->d_table = nullptr;
  h->d_epart = h->d_gpart = h->d_theta = h->d_E = h->d_grad = h->d_coeffs = h->d_ssum = nullptr;
  h->Bcap = 0;
  const size_t N = 1ull << h->n;
  const int G = blocks_per_state(h);
  rc = check_hip(hipMalloc(&h->d_phi, (size_t)B * N * sizeof(double2)), "hipMalloc(vqe phi)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_lam, (size_t)B * N * sizeof(double2)), "hipMalloc(vqe lambda)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_epart, (size_t)B * G * sizeof(double)), "hipMalloc(vqe epart)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_gpart, (size_t)B * std::max(1, h->nslots) * G * sizeof(double)), "hipMalloc(vqe gpart)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_theta, (size_t)B * std::max(1, h->P) * sizeof(double)), "hipMalloc(vqe theta)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_E, (size_t)B * sizeof(double)), "hipMalloc(vqe E)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_grad, (size_t)B * std::max(1, h->P) * sizeof(double)), "hipMalloc(vqe grad)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_coeffs, (size_t)B * std::max(1, h->nterms) * sizeof(double)), "hipMalloc(vqe coeffs)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_table, (size_t)B * std::max(1, h->nops) * 8 * sizeof(double2)), "hipMalloc(vqe table)");
  if (!rc) rc = check_hip(hipMalloc(&h->d_ssum, (size_t)B * std::max(1, h->nslots) * sizeof(double)), "hipMalloc(vqe slot sums)");
  if (rc) return rc;
  h->Bcap = B;
  return NWQ_OK;
}

// The per-gate schedule for B states on stream s (captured into a graph by
// the batched path, launched directly by the per-circuit path).
static int launch_global(nwq_vqe* h, int B, const double* theta, const double* coeffs, double* E, double* grad,
                         hipStream_t s) {
  const int G = blocks_per_state(h);
  const dim3 grid(G, B);
  hipLaunchKernelGGL(k_vqe_init, grid, dim3(kVqeBlock), 0, s, h->d_phi, h->n);
  for (int i = 0; i < h->nops; ++i)
    hipLaunchKernelGGL(k_vqe_gate, grid, dim3(kVqeBlock), 0, s, h->d_phi, h->n, h->ops[i], h->d_fixed, theta, h->P, 0);
  hipLaunchKernelGGL(k_vqe_hphi, grid, dim3(kVqeBlock), 0, s, h->d_phi, h->d_lam, h->n, h->d_terms, h->nterms,
                     coeffs, h->d_epart, grad != nullptr ? 1 : 0);
  if (grad != nullptr) {
    for (int i = h->nops - 1; i >= 0; --i) {
      const VqeOp& op = h->ops[i];
      if (op.slot >= 0) {
        hipLaunchKernelGGL(k_vqe_adjoint, grid, dim3(kVqeBlock), 0, s, h->d_phi, h->d_lam, h->n, op, h->d_fixed,
                           theta, h->P, h->nslots, h->d_gpart);
      } else {
        hipLaunchKernelGGL(k_vqe_gate, grid, dim3(kVqeBlock), 0, s, h->d_phi, h->n, op, h->d_fixed, theta, h->P, 1);
        hipLaunchKernelGGL(k_vqe_gate, grid, dim3(kVqeBlock), 0, s, h->d_lam, h->n, op, h->d_fixed, theta, h->P, 1);
      }
    }
  }
  if (grad != nullptr && h->nslots > 0)
    hipLaunchKernelGGL(k_vqe_slot_sums, dim3((h->nslots + kFinBlock / kWave - 1) / (kFinBlock / kWave), B),
                       dim3(kFinBlock), 0, s, h->d_gpart, G, h->nslots, h->d_ssum);
  hipLaunchKernelGGL(k_vqe_finish, dim3(B), dim3(kFinBlock), 0, s, h->d_epart, G, h->nslots,
                     h->d_slot_param, h->P, h->d_ssum, E, grad);
  return check_hip(hipGetLastError(), "vqe per-gate schedule");
}

// Fused program: blocks over the ops at tile width fused_k, forward phases for
// the register-blocked kernel, backward ops in reverse per block (chunks of
// at most kBwdMaxOps).
// Low tile bits of the fused schedule's blocks (clamped to [k - 8, k - 2] at
// width k).  A batch of 2^20-amplitude states at n=20 plans the HEA ansatz
// (L=8) into 26 backward blocks of width 11 with 6 low bits and 18 with 3; the
// shorter runs cost less than the passes they save (n=20, L=8, B=256: 129 ->
// 119 ms per batch).
constexpr int kVqeLowBits = 3;

static int build_fused(nwq_vqe* h) {
  if (h->fused_built) return NWQ_OK;
  const int low = h->low_bits > 0 ? h->low_bits : kVqeLowBits;
  const int n = h->n;
  std::vector<PGate> g(h->nops);
  for (int i = 0; i < h->nops; ++i) {
    const VqeOp& op = h->ops[i];
    const bool two = op.kind == OP_RZZ || op.kind == OP_CX || op.kind == OP_CZ || op.kind == OP_SWAP;
    g[i] = PGate{0, {op.q0, two ? op.q1 : -1}, two ? 2 : 1, {0, 0, 0}};
  }
  const int k = std::min(h->fused_k, n);
  const std::vector<Block> blocks = plan_blocks(g, n, std::max(k, 6), low);
  if (blocks.empty() && h->nops > 0) return set_error(NWQ_EINVAL, "fusion planner made no progress");
  std::vector<FusedPhase> phases;
  std::vector<FusedOp> fops;
  std::vector<VqeBwdOp> bops;
  h->fwd_blocks.clear();
  h->bwd_blocks.clear();
  h->bwd_tile0.clear();
  std::vector<Block> padded(blocks);
  for (Block& b : padded) pad_block(b, n, std::max(k, 8));
  size_t max_bwd_lds = 0;
  for (const Block& b : padded) {
    const int kb = b.c + b.m;
    if (kb < 8) return set_error(NWQ_EINVAL, "fused VQE path needs tiles of at least 2^8 amplitudes");
    std::vector<std::array<int, 4>> lb(g.size());
    std::vector<int> nq(g.size(), 1);
    for (int gi : b.gates) {
      lb[gi] = {local_bit(b, g[gi].q[0]), g[gi].nq == 2 ? local_bit(b, g[gi].q[1]) : 0};
      nq[gi] = g[gi].nq;
    }
    FusedBlockDev d{};
    d.c = b.c;
    d.m = b.m;
    for (int i = 0; i < b.m; ++i) d.hi[i] = b.hi[i];
    d.op_begin = (int)phases.size();
    for (const Phase& ph : plan_phases(b.gates, lb, nq, kb, b.c, h->fused_rbits)) {
      FusedPhase fp{};
      for (int i = 0; i < 4; ++i) fp.reg[i] = ph.reg[i] < 0 ? 0 : ph.reg[i];
      fp.op_begin = (int)fops.size();
      auto ridx = [&](int bit) {
        for (int i = 0; i < h->fused_rbits; ++i)
          if (ph.reg[i] == bit) return i;
        return -1;
      };
      for (int gi : ph.gates) {
        const VqeOp& op = h->ops[gi];
        FusedOp f{};
        f.mat = 8 * gi;
        const int r0 = ridx(lb[gi][0]), r1 = nq[gi] == 2 ? ridx(lb[gi][1]) : 0;
        f.lo = r0;
        if (op.kind == OP_ROT && op.axis == 2) {
          f.kind = 6;   // RZ: diagonal of its 2x2 table entry
        } else if (op.kind == OP_ROT || op.kind == OP_FIX1) {
          f.kind = 0;
          // RX: M[0][0] = cos(theta / 2) is real for every theta; RY: all of M is
          f.real00 = op.kind == OP_ROT ? (op.axis == 1 ? 2 : 1) : 0;
        } else if (op.kind == OP_RZZ || op.kind == OP_CZ) {
          f.kind = 4; f.o0 = r0; f.o1 = r1;
        } else if (op.kind == OP_CX) {
          f.kind = 3; f.o0 = r0; f.o1 = r1;
        } else {
          f.kind = 5; f.o0 = r0; f.o1 = r1;
        }
        f.code = rb_op_code(f);
        fops.push_back(f);
      }
      fp.op_count = (int)fops.size() - fp.op_begin;
      fill_phase_offsets(fp, h->fused_rbits, nullptr, nullptr);
      phases.push_back(fp);
    }
    d.op_count = (int)phases.size() - d.op_begin;
    fill_entry_offsets(d, h->fused_rbits);
    set_direct_io(d, phases[d.op_begin], phases.back(), h->fused_rbits);
    h->fwd_blocks.push_back(d);
  }
  // Backward: register-blocked with 3 register bits when every tile gives at
  // least one full wave (2^(k-3) >= 64), else one LDS pass per gate.
  constexpr int kBwdBits = 3;
  // The backward sweep plans its own blocks when the forward width exceeds
  // what its kernels take (tiles of at most 2^11: 256 threads x 8 amplitudes):
  // any partition of the reversed gate list gives the same sweep.
  std::vector<Block> bpadded;
  const int kbw = std::min(k, kBwdMaxTileBits);
  if (kbw == k) {
    bpadded = padded;
  } else {
    bpadded = plan_blocks(g, n, std::max(kbw, 6), low);
    if (bpadded.empty() && h->nops > 0) return set_error(NWQ_EINVAL, "fusion planner made no progress");
    for (Block& b : bpadded) pad_block(b, n, std::max(kbw, 8));
  }
  for (const Block& b : bpadded) max_bwd_lds = std::max(max_bwd_lds, (size_t)2 * sizeof(double2) << (b.c + b.m));
  h->bwd_rb = true;
  for (const Block& b : bpadded) h->bwd_rb = h->bwd_rb && (b.c + b.m) - kBwdBits >= 6;
  std::vector<VqeBwdRop> rops;
  for (auto bit = bpadded.rbegin(); h->bwd_rb && bit != bpadded.rend(); ++bit) {
    const Block& b = *bit;
    const int kb = b.c + b.m;
    std::vector<std::array<int, 4>> lb(g.size());
    std::vector<int> nq(g.size(), 1);
    std::vector<int> rev(b.gates.rbegin(), b.gates.rend());
    for (int gi : rev) {
      lb[gi] = {local_bit(b, g[gi].q[0]), g[gi].nq == 2 ? local_bit(b, g[gi].q[1]) : 0};
      nq[gi] = g[gi].nq;
    }
    for (size_t s0 = 0; s0 < rev.size(); s0 += kBwdMaxOps) {
      const std::vector<int> chunk(rev.begin() + s0, rev.begin() + std::min(rev.size(), s0 + kBwdMaxOps));
      FusedBlockDev d{};
      d.c = b.c;
      d.m = b.m;
      for (int i = 0; i < b.m; ++i) d.hi[i] = b.hi[i];
      d.op_begin = (int)phases.size();
      for (const Phase& ph : plan_phases(chunk, lb, nq, kb, 0, kBwdBits)) {
        FusedPhase fp{};
        for (int i = 0; i < 4; ++i) fp.reg[i] = ph.reg[i] < 0 ? 0 : ph.reg[i];
        fp.op_begin = (int)rops.size();
        auto ridx = [&](int bit) {
          for (int i = 0; i < kBwdBits; ++i)
            if (ph.reg[i] == bit) return i;
          return -1;
        };
        std::vector<VqeBwdRop> pops;
        for (int gi : ph.gates) {
          const VqeOp& op = h->ops[gi];
          VqeBwdRop o{};
          o.r0 = ridx(lb[gi][0]);
          o.r1 = nq[gi] == 2 ? ridx(lb[gi][1]) : 0;
          o.axis = op.axis;
          o.slot = op.slot;
          o.mat = 8 * gi + 4;
          o.kind = op.kind == OP_ROT ? 0 : op.kind == OP_RZZ ? 1 : op.kind == OP_FIX1 ? 2 : op.kind == OP_CX ? 3
                 : op.kind == OP_CZ ? 4 : 5;
          o.code = bwd_rop_code(o);
          pops.push_back(o);
        }
        int ld_perm[16], st_perm[16];
        fold_permutations(
            pops, kBwdBits, [](const VqeBwdRop& o) { return o.kind == 3 || o.kind == 5; },
            [](const VqeBwdRop& o) {
              return (o.kind == 0 || o.kind == 2) ? (1u << o.r0) : ((1u << o.r0) | (1u << o.r1));
            },
            [](const VqeBwdRop& o, int j) { return o.kind == 3 ? reg_cx(o.r0, o.r1, j) : reg_swap(o.r0, o.r1, j); },
            ld_perm, st_perm);
        rops.insert(rops.end(), pops.begin(), pops.end());
        fp.op_count = (int)rops.size() - fp.op_begin;
        fill_phase_offsets(fp, kBwdBits, ld_perm, st_perm);
        phases.push_back(fp);
      }
      d.op_count = (int)phases.size() - d.op_begin;
      fill_entry_offsets(d, kBwdBits);
      h->bwd_blocks.push_back(d);
      h->bwd_tile0.push_back(bit + 1 == bpadded.rend() ? 1 : 0);
    }
  }
  for (auto bit = bpadded.rbegin(); !h->bwd_rb && bit != bpadded.rend(); ++bit) {
    const Block& b = *bit;
    std::vector<VqeBwdOp> rev;
    for (auto it = b.gates.rbegin(); it != b.gates.rend(); ++it) {
      const int gi = *it;
      const VqeOp& op = h->ops[gi];
      VqeBwdOp o{};
      o.b0 = local_bit(b, op.q0);
      o.b1 = g[gi].nq == 2 ? local_bit(b, op.q1) : 0;
      o.lo = g[gi].nq == 2 ? std::min(o.b0, o.b1) : o.b0;
      o.hi = g[gi].nq == 2 ? std::max(o.b0, o.b1) : 0;
      o.axis = op.axis;
      o.slot = op.slot;
      o.mat = 8 * gi + 4;
      o.kind = op.kind == OP_ROT ? 0 : op.kind == OP_RZZ ? 1 : op.kind == OP_FIX1 ? 2 : op.kind == OP_CX ? 3
             : op.kind == OP_CZ ? 4 : 5;
      rev.push_back(o);
    }
    for (size_t s0 = 0; s0 < rev.size(); s0 += kBwdMaxOps) {
      FusedBlockDev d{};
      d.c = b.c;
      d.m = b.m;
      for (int i = 0; i < b.m; ++i) d.hi[i] = b.hi[i];
      d.op_begin = (int)bops.size();
      const size_t e = std::min(rev.size(), s0 + kBwdMaxOps);
      for (size_t i = s0; i < e; ++i) bops.push_back(rev[i]);
      d.op_count = (int)(e - s0);
      h->bwd_blocks.push_back(d);
      h->bwd_tile0.push_back(bit + 1 == bpadded.rend() ? 1 : 0);
    }
  }
  // lambda = H phi: the first pass takes tiles of the low kt bits with every
  // diagonal term and the terms whose flipped bits lie there; further passes
  // take tiles of the 6 low bits plus up to kt - 6 high bits, greedily, for
  // the remaining terms; terms needing more high bits than that go to a
  // gather pass.  Tiles are widened to 2^kt entries with unused high bits.
  std::vector<HTerm> hterms;
  std::vector<int> widx;
  h->hlaunch.clear();
  {
    const int kt = std::min(n, kHTileBits);
    std::vector<int> diag, rest, wide;
    for (int t = 0; t < h->nterms; ++t) {
      const unsigned long long x = h->terms[t].x;
      if (x == 0) diag.push_back(t);
      else if ((x >> kt) == 0) rest.push_back(t);   // in the first pass
      else if (__builtin_popcountll(x >> 6) > kt - 6) wide.push_back(t);
      else rest.push_back(t);
    }
    auto add_pass = [&](int c, std::vector<int> hi, const std::vector<int>& dg, const std::vector<int>& fl) {
      for (int q = c; q < n && (int)hi.size() < kt - c; ++q)
        if (std::find(hi.begin(), hi.end(), q) == hi.end()) hi.push_back(q);
      std::sort(hi.begin(), hi.end());
      auto local = [&](unsigned long long mask) {
        unsigned l = (unsigned)(mask & ((1ull << c) - 1ull));
        for (size_t i = 0; i < hi.size(); ++i)
          if ((mask >> hi[i]) & 1ull) l |= 1u << (c + i);
        return l;
      };
      unsigned long long inside = (1ull << c) - 1ull;
      for (int q : hi) inside |= 1ull << q;
      std::vector<int> all(dg);
      all.insert(all.end(), fl.begin(), fl.end());
      for (size_t s0 = 0; s0 < all.size(); s0 += kHMaxTerms) {
        nwq_vqe::HLaunch L{};
        L.p.c = c;
        L.p.m = (int)hi.size();
        for (size_t i = 0; i < hi.size(); ++i) L.p.hi[i] = hi[i];
        L.p.t_begin = (int)hterms.size();
        for (size_t i = s0; i < std::min(all.size(), s0 + kHMaxTerms); ++i) {
          const VqeTerm& T = h->terms[all[i]];
          const int pc = __builtin_popcountll(T.x & T.z);
          hterms.push_back(HTerm{local(T.x), local(T.z & inside), T.z & ~inside, pc & 3, pc & 1, all[i], 0});
          if (T.x == 0) ++L.p.n_diag;
          else ++L.p.n_flip;
        }
        h->hlaunch.push_back(L);
      }
    };
    std::vector<int> first_flips, later;
    for (int t : rest) ((h->terms[t].x >> kt) == 0 ? first_flips : later).push_back(t);
    add_pass(kt, {}, diag, first_flips);
    const int c = std::min(6, kt);
    while (!later.empty()) {
      std::vector<int> hi, take, keep;
      for (int t : later) {
        std::vector<int> need;
        for (int q = c; q < n; ++q)
          if (((h->terms[t].x >> q) & 1ull) && std::find(hi.begin(), hi.end(), q) == hi.end()) need.push_back(q);
        if ((int)(hi.size() + need.size()) <= kt - c) {
          hi.insert(hi.end(), need.begin(), need.end());
          take.push_back(t);
        } else {
          keep.push_back(t);
        }
      }
      add_pass(c, hi, {}, take);
      later.swap(keep);
    }
    if (!wide.empty()) {
      nwq_vqe::HLaunch L{};
      L.wide = 1;
      L.w_begin = 0;
      L.w_count = (int)wide.size();
      widx = wide;
      h->hlaunch.push_back(L);
    }
    for (size_t i = 0; i < h->hlaunch.size(); ++i) {
      h->hlaunch[i].p.first = i == 0;
      h->hlaunch[i].p.last = i + 1 == h->hlaunch.size();
    }
  }
  const size_t ph_bytes = phases.size() * sizeof(FusedPhase);
  h->fused_ops_off = (ph_bytes + 255) & ~size_t(255);
  h->fused_bwd_off = (h->fused_ops_off + fops.size() * sizeof(FusedOp) + 255) & ~size_t(255);
  h->fused_rop_off = (h->fused_bwd_off + bops.size() * sizeof(VqeBwdOp) + 255) & ~size_t(255);
  h->fused_hterm_off = (h->fused_rop_off + rops.size() * sizeof(VqeBwdRop) + 255) & ~size_t(255);
  h->fused_widx_off = (h->fused_hterm_off + hterms.size() * sizeof(HTerm) + 255) & ~size_t(255);
  const size_t total = h->fused_widx_off + widx.size() * sizeof(int) + 16;
  std::vector<char> prog(total, 0);
  if (!phases.empty()) std::memcpy(prog.data(), phases.data(), ph_bytes);
  if (!fops.empty()) std::memcpy(prog.data() + h->fused_ops_off, fops.data(), fops.size() * sizeof(FusedOp));
  if (!bops.empty()) std::memcpy(prog.data() + h->fused_bwd_off, bops.data(), bops.size() * sizeof(VqeBwdOp));
  if (!rops.empty()) std::memcpy(prog.data() + h->fused_rop_off, rops.data(), rops.size() * sizeof(VqeBwdRop));
  if (!hterms.empty()) std::memcpy(prog.data() + h->fused_hterm_off, hterms.data(), hterms.size() * sizeof(HTerm));
  if (!widx.empty()) std::memcpy(prog.data() + h->fused_widx_off, widx.data(), widx.size() * sizeof(int));
  // dynamic LDS above 64 KiB is enabled here, outside any graph capture
  const int kbt = std::min(std::min(h->fused_k, kBwdMaxTileBits), n);
  const size_t max_rb_lds = 2 * bwd_rb_tile_bytes(kbt < 8 ? 8 : kbt);
  if (max_bwd_lds > (size_t)kMaxDynamicLds || max_rb_lds > (size_t)kMaxDynamicLds ||
      sizeof(double2) * hpad(1u << kHTileBits) > (size_t)kMaxDynamicLds)
    return set_error(NWQ_EINVAL, "VQE tile larger than the dynamic LDS limit");
  int rc = enable_dynamic_lds((const void*)k_vqe_bwd_tile);
  for (const void* f : {(const void*)k_vqe_hphi_tile<false, false>, (const void*)k_vqe_hphi_tile<true, false>,
                        (const void*)k_vqe_hphi_tile<false, true>, (const void*)k_vqe_hphi_tile<true, true>,
                        (const void*)k_vqe_bwd_rb<3, false>, (const void*)k_vqe_bwd_rb<3, true>})
    if (!rc) rc = enable_dynamic_lds(f);
  if (!rc) rc = fused_rb_enable_lds();
  if (!rc) rc = check_hip(hipMalloc(&h->d_fused, total), "hipMalloc(vqe fused program)");
  if (!rc) rc = check_hip(hipMemcpy(h->d_fused, prog.data(), total, hipMemcpyHostToDevice), "hipMemcpy(vqe fused program)");
  if (rc) return rc;
  h->fused_built = true;
  h->fused_bytes = total;
  return NWQ_OK;
}

static int fused_grid(const nwq_vqe* h) {
  // workgroups per state, shared by the forward and backward launches (the
  // gradient partials have one slot per workgroup): sized on the backward tiles
  const int k = std::min(std::max(std::min(h->fused_k, kBwdMaxTileBits), 8), h->n);
  const unsigned long long ntiles = 1ull << (h->n - k);
  return (int)std::max<unsigned long long>(1, std::min<unsigned long long>(ntiles, blocks_per_state(h)));
}

static int launch_fused(nwq_vqe* h, int B, const double* theta, const double* coeffs, double* E, double* grad,
                        hipStream_t s) {
  int rc = build_fused(h);
  if (rc) return rc;
  const int G = fused_grid(h);
  const dim3 grid(G, B);
  const FusedPhase* dph = static_cast<const FusedPhase*>(h->d_fused);
  const FusedOp* dfo = reinterpret_cast<const FusedOp*>(static_cast<char*>(h->d_fused) + h->fused_ops_off);
  const VqeBwdOp* dbo = reinterpret_cast<const VqeBwdOp*>(static_cast<char*>(h->d_fused) + h->fused_bwd_off);
  const int stride = 8 * h->nops;
  hipLaunchKernelGGL(k_vqe_init, grid, dim3(kVqeBlock), 0, s, h->d_phi, h->n);
  hipLaunchKernelGGL(k_vqe_mats, dim3((h->nops + 255) / 256, B), dim3(256), 0, s, h->d_ops, h->nops, h->d_fixed,
                     theta, h->P, h->d_table);
  // phi starts at |0...0>: amplitudes can be nonzero only where every qubit no
  // earlier block touched is zero, and a block maps each tile to itself and
  // zero tiles to zero, so each block runs only the tiles whose index is zero
  // on its non-tile qubits outside that support (the first block: tile 0)
  unsigned long long support = 0;
  for (size_t bi = 0; bi < h->fwd_blocks.size(); ++bi) {
    const FusedBlockDev& d = h->fwd_blocks[bi];
    unsigned long long tiles_of = 0, tile_mask = 0;
    for (int q = 0; q < d.c; ++q) tiles_of |= 1ull << q;
    for (int i = 0; i < d.m; ++i) tiles_of |= 1ull << d.hi[i];
    for (int q = 0, j = 0; q < h->n; ++q) {
      if ((tiles_of >> q) & 1ull) continue;
      if ((support >> q) & 1ull) tile_mask |= 1ull << j;
      ++j;
    }
    support |= tiles_of;
    launch_fused_rb(s, h->d_phi, h->n, d, dph, dfo, h->d_table, h->fused_rbits, B, stride, G, h->fused_flags, 0,
                    tile_mask);
  }
  const HTerm* dht = reinterpret_cast<const HTerm*>(static_cast<char*>(h->d_fused) + h->fused_hterm_off);
  const int* dwi = reinterpret_cast<const int*>(static_cast<char*>(h->d_fused) + h->fused_widx_off);
  for (const auto& L : h->hlaunch) {
    const int sel = (L.p.first ? 1 : 0) | (L.p.last ? 2 : 0);
    if (L.wide) {
      auto kw = sel == 0 ? k_vqe_hphi_wide<false, false> : sel == 1 ? k_vqe_hphi_wide<true, false>
              : sel == 2 ? k_vqe_hphi_wide<false, true> : k_vqe_hphi_wide<true, true>;
      hipLaunchKernelGGL(kw, grid, dim3(kVqeBlock), 0, s, h->d_phi, h->d_lam, h->n, h->d_terms, dwi + L.w_begin,
                         L.w_count, h->nterms, coeffs, h->d_epart);
    } else {
      auto kt = sel == 0 ? k_vqe_hphi_tile<false, false> : sel == 1 ? k_vqe_hphi_tile<true, false>
              : sel == 2 ? k_vqe_hphi_tile<false, true> : k_vqe_hphi_tile<true, true>;
      const size_t lds = sizeof(double2) * hpad(1u << (L.p.c + L.p.m));
      hipLaunchKernelGGL(kt, grid, dim3(kHBlock), lds, s, h->d_phi, h->d_lam, h->n, L.p, dht, h->d_terms, h->nterms,
                         coeffs, h->d_epart);
    }
  }
  if (grad != nullptr) {
    const VqeBwdRop* dro = reinterpret_cast<const VqeBwdRop*>(static_cast<char*>(h->d_fused) + h->fused_rop_off);
    for (size_t bi = 0; bi < h->bwd_blocks.size(); ++bi) {
      const FusedBlockDev& d = h->bwd_blocks[bi];
      const int kb = d.c + d.m;
      const unsigned long long nt = h->bwd_tile0[bi] ? 1ull : 1ull << (h->n - kb);
      if (h->bwd_rb) {
        if (h->fused_flags & kFusedNonTemporal)
          hipLaunchKernelGGL((k_vqe_bwd_rb<3, true>), grid, dim3(1u << (kb - 3)), 2 * bwd_rb_tile_bytes(kb), s,
                             h->d_phi, h->d_lam, h->n, d, dph, dro, h->d_table, stride, h->nslots, h->d_gpart, nt);
        else
          hipLaunchKernelGGL((k_vqe_bwd_rb<3, false>), grid, dim3(1u << (kb - 3)), 2 * bwd_rb_tile_bytes(kb), s,
                             h->d_phi, h->d_lam, h->n, d, dph, dro, h->d_table, stride, h->nslots, h->d_gpart, nt);
      } else {
        const size_t lds = 2 * sizeof(double2) << kb;
        hipLaunchKernelGGL(k_vqe_bwd_tile, grid, dim3(kBwdBlock), lds, s, h->d_phi, h->d_lam, h->n, d, dbo,
                           h->d_table, stride, h->nslots, h->d_gpart, nt);
      }
    }
  }
  if (grad != nullptr && h->nslots > 0)
    hipLaunchKernelGGL(k_vqe_slot_sums, dim3((h->nslots + kFinBlock / kWave - 1) / (kFinBlock / kWave), B),
                       dim3(kFinBlock), 0, s, h->d_gpart, G, h->nslots, h->d_ssum);
  hipLaunchKernelGGL(k_vqe_finish, dim3(B), dim3(kFinBlock), 0, s, h->d_epart, G, h->nslots,
                     h->d_slot_param, h->P, h->d_ssum, E, grad);
  return check_hip(hipGetLastError(), "vqe fused schedule");
}

static int run_graph(nwq_vqe* h, int B, bool want_grad, bool with_coeffs) {
  const bool fused = h->cfg.mode == 3 || (h->cfg.mode == 0 && h->n > 12);
  const auto key = std::make_pair(B, (want_grad ? 1 : 0) | (with_coeffs ? 2 : 0) | (fused ? 4 : 0));
  auto it = h->graphs.find(key);
  if (it == h->graphs.end()) {
    if (fused) {
      const int rcb = build_fused(h);   // host planning and program upload stay outside the capture
      if (rcb) return rcb;
    }
    int rc = check_hip(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (rc) return rc;
    if (fused)
      rc = launch_fused(h, B, h->d_theta, with_coeffs ? h->d_coeffs : nullptr, h->d_E, want_grad ? h->d_grad : nullptr,
                        h->stream);
    else
      rc = launch_global(h, B, h->d_theta, with_coeffs ? h->d_coeffs : nullptr, h->d_E, want_grad ? h->d_grad : nullptr,
                         h->stream);
    hipGraph_t g = nullptr;
    const int rc2 = check_hip(hipStreamEndCapture(h->stream, &g), "hipStreamEndCapture");
    if (rc) return rc;
    if (rc2) return rc2;
    hipGraphExec_t ex = nullptr;
    rc = check_hip(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    (void)hipGraphDestroy(g);
    if (rc) return rc;
    it = h->graphs.emplace(key, ex).first;
  }
  return check_hip(hipGraphLaunch(it->second, h->stream), "hipGraphLaunch");
}

}  // namespace nwq

using namespace nwq;

extern "C" {

int nwq_vqe_create(int n, int n_ops, const int* types, const int* qubits, const int* params, int n_params,
                   int n_terms, const uint64_t* xmask, const uint64_t* zmask, const double* coeffs, void* stream,
                   nwq_vqe_handle* out) {
  if (!out) return vqe_fail(NWQ_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  if (n < 1 || n > 30) return vqe_fail(NWQ_ERANGE, "VQE register must have 1..30 qubits");
  if (n_ops < 0 || (n_ops > 0 && (!types || !qubits || !params))) return vqe_fail(NWQ_EINVAL, "bad op arrays");
  if (n_terms < 0 || (n_terms > 0 && (!xmask || !zmask || !coeffs))) return vqe_fail(NWQ_EINVAL, "bad term arrays");
  if (n_params < 0) return vqe_fail(NWQ_EINVAL, "negative parameter count");
  std::unique_ptr<nwq_vqe> h(new nwq_vqe());
  h->n = n;
  h->P = n_params;
  h->user_stream = static_cast<hipStream_t>(stream);
  std::vector<double2> fixed;
  for (int i = 0; i < n_ops; ++i) {
    const int t = types[i], a = qubits[2 * i], b = qubits[2 * i + 1], p = params[i];
    VqeOp op{};
    op.q0 = a;
    op.q1 = b;
    op.param = -1;
    op.slot = -1;
    op.mat = -1;
    const bool two = t == NWQ_GATE_CX || t == NWQ_GATE_CZ || t == NWQ_GATE_SWAP || t == NWQ_GATE_RZZ;
    if (a < 0 || a >= n || (two && (b < 0 || b >= n))) return vqe_fail(NWQ_ERANGE, "op " + std::to_string(i) + ": qubit out of range");
    if (two && a == b) return vqe_fail(NWQ_EDUP, "op " + std::to_string(i) + ": repeated qubit");
    const bool param = t == NWQ_GATE_RX || t == NWQ_GATE_RY || t == NWQ_GATE_RZ || t == NWQ_GATE_RZZ;
    if (param) {
      if (p < 0 || p >= n_params) return vqe_fail(NWQ_EINVAL, "op " + std::to_string(i) + ": parameter index out of range");
      op.param = p;
      op.slot = h->nslots++;
      h->slot_param.push_back(p);
      if (t == NWQ_GATE_RZZ) {
        op.kind = OP_RZZ;
      } else {
        op.kind = OP_ROT;
        op.axis = t == NWQ_GATE_RX ? 0 : (t == NWQ_GATE_RY ? 1 : 2);
      }
    } else if (t == NWQ_GATE_CX) {
      op.kind = OP_CX;
    } else if (t == NWQ_GATE_CZ) {
      op.kind = OP_CZ;
    } else if (t == NWQ_GATE_SWAP) {
      op.kind = OP_SWAP;
    } else if (t >= NWQ_GATE_I && t <= NWQ_GATE_TDG) {
      if (t == NWQ_GATE_I) continue;
      cd m[16];
      gate_matrix(t, nullptr, m);
      op.kind = OP_FIX1;
      op.mat = (int)(fixed.size() / 8);
      for (int k = 0; k < 4; ++k) fixed.push_back(make_double2(m[k].real(), m[k].imag()));
      const int tr[4] = {0, 2, 1, 3};   // U^dag = conj(U^T)
      for (int k = 0; k < 4; ++k) fixed.push_back(make_double2(m[tr[k]].real(), -m[tr[k]].imag()));
    } else {
      return vqe_fail(NWQ_EINVAL, "op " + std::to_string(i) + ": gate type not supported in a VQE program");
    }
    h->ops.push_back(op);
  }
  h->nops = (int)h->ops.size();
  std::vector<VqeTerm> terms(n_terms);
  const unsigned long long all = (1ull << n) - 1ull;
  for (int t = 0; t < n_terms; ++t) {
    if ((xmask[t] & ~all) || (zmask[t] & ~all)) return vqe_fail(NWQ_ERANGE, "Pauli mask has bits beyond n");
    if (!std::isfinite(coeffs[t])) return vqe_fail(NWQ_EINVAL, "non-finite coefficient");
    terms[t] = VqeTerm{xmask[t], zmask[t], coeffs[t], __builtin_popcountll(xmask[t] & zmask[t]) & 3, 0};
  }
  h->nterms = n_terms;
  h->terms = terms;
  int rc = check_hip(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking), "hipStreamCreate");
  if (!rc) rc = check_hip(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming), "hipEventCreate");
  if (!rc) rc = check_hip(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming), "hipEventCreate");
  auto up = [&](void** dst, const void* src, size_t bytes) -> int {
    const size_t b = std::max<size_t>(bytes, 16);
    int r = check_hip(hipMalloc(dst, b), "hipMalloc(vqe program)");
    if (r) return r;
    h->program_bytes += b;
    if (bytes) r = check_hip(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy(vqe program)");
    return r;
  };
  if (!rc) rc = up((void**)&h->d_ops, h->ops.data(), h->ops.size() * sizeof(VqeOp));
  if (!rc) rc = up((void**)&h->d_fixed, fixed.data(), fixed.size() * sizeof(double2));
  if (!rc) rc = up((void**)&h->d_terms, terms.data(), terms.size() * sizeof(VqeTerm));
  if (!rc) rc = up((void**)&h->d_slot_param, h->slot_param.data(), h->slot_param.size() * sizeof(int));
  if (rc) {
    nwq_vqe_destroy(h.release());
    return rc;
  }
  h->cfg.threads = n <= 8 ? 128 : 256;
  *out = h.release();
  return NWQ_OK;
}

int nwq_vqe_destroy(nwq_vqe_handle h) {
  if (!h) return NWQ_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  for (void* p : {(void*)h->d_ops, (void*)h->d_fixed, (void*)h->d_terms, (void*)h->d_slot_param, (void*)h->d_phi,
                  (void*)h->d_lam, (void*)h->d_epart, (void*)h->d_gpart, (void*)h->d_theta, (void*)h->d_E,
                  (void*)h->d_grad, (void*)h->d_coeffs, (void*)h->d_table, (void*)h->d_ssum, h->d_fused})
    if (p) (void)hipFree(p);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  if (h->ev_out) (void)hipEventDestroy(h->ev_out);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return NWQ_OK;
}

int nwq_vqe_memory(nwq_vqe_handle h, int B, size_t* held, size_t* at_B) {
  if (!h) return vqe_fail(NWQ_EINVAL, "NULL handle");
  if (B < 0 || B > 65535) return vqe_fail(NWQ_EINVAL, "batch size must be in [0, 65535]");
  const size_t per = global_bytes_per_vector(h);
  const size_t base = h->program_bytes + h->fused_bytes;
  if (held) *held = base + (size_t)h->Bcap * per;
  if (at_B) {
    // the LDS-resident path keeps no per-vector buffers; every other path
    // grows the capacity to B (never shrinks it)
    const bool lds = h->cfg.mode == 1 || (h->cfg.mode == 0 && lds_fits(h, h->cfg.threads, true));
    const size_t cap = lds ? (size_t)h->Bcap : std::max<size_t>(h->Bcap, (size_t)B);
    *at_B = base + cap * per;
  }
  return NWQ_OK;
}

int nwq_vqe_info(nwq_vqe_handle h, int* n_params, int* n_ops, int* n_slots) {
  if (!h) return vqe_fail(NWQ_EINVAL, "NULL handle");
  if (n_params) *n_params = h->P;
  if (n_ops) *n_ops = h->nops;
  if (n_slots) *n_slots = h->nslots;
  return NWQ_OK;
}

int nwq_vqe_set_config(nwq_vqe_handle h, int mode, int threads, int blocks_per_state_) {
  if (!h) return vqe_fail(NWQ_EINVAL, "NULL handle");
  if (mode < 0 || mode > 3) return vqe_fail(NWQ_EINVAL, "mode must be 0 (auto), 1 (LDS), 2 (per-gate) or 3 (fused)");
  if (mode == 3 && h->n < 8) return vqe_fail(NWQ_EINVAL, "the fused path needs n >= 8");
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
    return vqe_fail(NWQ_EINVAL, "threads must be 64, 128, 256, 512 or 1024");
  if (blocks_per_state_ < 0 || blocks_per_state_ > 4096) return vqe_fail(NWQ_EINVAL, "blocks per state in [0, 4096]");
  if (mode == 1 && h->n > 12) return vqe_fail(NWQ_EINVAL, "the LDS-resident path holds n <= 12");
  if (blocks_per_state_ != h->cfg.blocks_per_state) {   // partial buffers and graphs depend on it
    (void)hipStreamSynchronize(h->stream);
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    h->cfg.blocks_per_state = blocks_per_state_;
    const int B = h->Bcap;
    h->Bcap = 0;
    if (B > 0) {
      const int rc = ensure_global(h, B);
      if (rc) return rc;
    }
  }
  h->cfg.mode = mode;
  h->cfg.threads = threads;
  return NWQ_OK;
}

int nwq_vqe_set_flags(nwq_vqe_handle h, int flags) {
  if (!h) return vqe_fail(NWQ_EINVAL, "NULL handle");
  if (flags < 0 || flags > 3) return vqe_fail(NWQ_EINVAL, "flags must be in [0, 3]");
  if (flags != h->fused_flags) {   // the captured schedules hold the kernels
    (void)hipStreamSynchronize(h->stream);
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    h->fused_flags = flags;
  }
  return NWQ_OK;
}

int nwq_vqe_set_lowbits(nwq_vqe_handle h, int c) {
  if (!h) return vqe_fail(NWQ_EINVAL, "NULL handle");
  if (c != 0 && (c < 3 || c > 8)) return vqe_fail(NWQ_EINVAL, "low tile bits must be 0 or in [3, 8]");
  if (c != h->low_bits) {   // the fused program is planned again on next use
    (void)hipStreamSynchronize(h->stream);
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    if (h->d_fused) (void)hipFree(h->d_fused);
    h->d_fused = nullptr;
    h->fused_built = false;
    h->fused_bytes = 0;
    h->low_bits = c;
  }
  return NWQ_OK;
}

int nwq_vqe_get_config(nwq_vqe_handle h, int* mode, int* threads, int* blocks_per_state_) {
  if (!h) return vqe_fail(NWQ_EINVAL, "NULL handle");
  if (mode) *mode = h->cfg.mode;
  if (threads) *threads = h->cfg.threads;
  if (blocks_per_state_) *blocks_per_state_ = blocks_per_state(h);
  return NWQ_OK;
}

static int eval_common(nwq_vqe_handle h, int B, const double* theta, const double* coeffs, double* E, double* grad,
                       bool single) {
  if (!h) return vqe_fail(NWQ_EINVAL, "NULL handle");
  if (B < 1 || B > 65535) return vqe_fail(NWQ_EINVAL, "batch size must be in [1, 65535]");
  if ((!theta && h->P > 0) || !E) return vqe_fail(NWQ_EINVAL, "NULL theta or energy pointer");
  int rc = check_hip(hipEventRecord(h->ev_in, h->user_stream), "hipEventRecord");
  if (!rc) rc = check_hip(hipStreamWaitEvent(h->stream, h->ev_in, 0), "hipStreamWaitEvent");
  if (rc) return rc;
  const bool want_grad = grad != nullptr;
  const int mode = single ? 2 : h->cfg.mode;
  const bool use_lds = !single && (mode == 1 || (mode == 0 && h->n <= 12 && lds_fits(h, h->cfg.threads, want_grad)));
  if (use_lds) {
    if (!lds_fits(h, h->cfg.threads, want_grad)) return vqe_fail(NWQ_EINVAL, "program does not fit the LDS-resident path");
    rc = launch_lds(h, B, theta, coeffs, E, grad, h->stream);
  } else if (single) {
    rc = ensure_global(h, B);
    if (!rc) rc = launch_global(h, B, theta, coeffs, E, grad, h->stream);
  } else {
    rc = ensure_global(h, B);
    if (!rc && h->P > 0)
      rc = check_hip(hipMemcpyAsync(h->d_theta, theta, (size_t)B * h->P * sizeof(double), hipMemcpyDeviceToDevice, h->stream),
                     "hipMemcpyAsync(theta)");
    if (!rc && coeffs && h->nterms > 0)
      rc = check_hip(hipMemcpyAsync(h->d_coeffs, coeffs, (size_t)B * h->nterms * sizeof(double), hipMemcpyDeviceToDevice,
                                    h->stream), "hipMemcpyAsync(coeffs)");
    if (!rc) rc = run_graph(h, B, want_grad, coeffs != nullptr);
    if (!rc) rc = check_hip(hipMemcpyAsync(E, h->d_E, (size_t)B * sizeof(double), hipMemcpyDeviceToDevice, h->stream),
                            "hipMemcpyAsync(E)");
    if (!rc && want_grad && h->P > 0)
      rc = check_hip(hipMemcpyAsync(grad, h->d_grad, (size_t)B * h->P * sizeof(double), hipMemcpyDeviceToDevice, h->stream),
                     "hipMemcpyAsync(grad)");
  }
  if (rc) return rc;
  rc = check_hip(hipEventRecord(h->ev_out, h->stream), "hipEventRecord");
  if (!rc) rc = check_hip(hipStreamWaitEvent(h->user_stream, h->ev_out, 0), "hipStreamWaitEvent");
  return rc;
}

int nwq_vqe_eval(nwq_vqe_handle h, int B, const double* theta_dev, double* energy_dev, double* grad_dev) {
  return eval_common(h, B, theta_dev, nullptr, energy_dev, grad_dev, false);
}

int nwq_vqe_eval_coeffs(nwq_vqe_handle h, int B, const double* theta_dev, const double* coeffs_dev,
                        double* energy_dev, double* grad_dev) {
  return eval_common(h, B, theta_dev, coeffs_dev, energy_dev, grad_dev, false);
}

int nwq_vqe_eval_single(nwq_vqe_handle h, const double* theta_dev, double* energy_dev, double* grad_dev) {
  return eval_common(h, 1, theta_dev, nullptr, energy_dev, grad_dev, true);
}

}  // extern "C"

extern "C" {

int nwq_vqe_autotune(nwq_vqe_handle h, int B, int with_grad, double* best_ms) {
  if (!h) return vqe_fail(NWQ_EINVAL, "NULL handle");
  if (B < 1 || B > 65535) return vqe_fail(NWQ_EINVAL, "batch size must be in [1, 65535]");
  double *theta = nullptr, *E = nullptr, *grad = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  const size_t P = std::max(1, h->P);
  int rc = check_hip(hipMalloc(&theta, (size_t)B * P * sizeof(double)), "hipMalloc(autotune theta)");
  if (!rc) rc = check_hip(hipMalloc(&E, (size_t)B * sizeof(double)), "hipMalloc(autotune E)");
  if (!rc) rc = check_hip(hipMalloc(&grad, (size_t)B * P * sizeof(double)), "hipMalloc(autotune grad)");
  if (!rc) rc = check_hip(hipMemsetAsync(theta, 0, (size_t)B * P * sizeof(double), h->stream), "hipMemsetAsync");
  if (!rc) rc = check_hip(hipEventCreate(&t0), "hipEventCreate");
  if (!rc) rc = check_hip(hipEventCreate(&t1), "hipEventCreate");
  struct Cand { int mode, threads, bps; };
  std::vector<Cand> cands;
  if (h->n <= 12)
    for (int t : {64, 128, 256, 512, 1024})
      if (lds_fits(h, t, with_grad != 0)) cands.push_back({1, t, 0});
  const unsigned long long pairs = 1ull << (h->n - 1);
  for (int bps : {0, 8, 16, 32, 64, 128, 256, 512, 1024})
    if (bps == 0 || (unsigned long long)bps * 256 <= pairs) cands.push_back({2, h->cfg.threads, bps});
  if (h->n >= 13)
    for (int bps : {0, 16, 32, 64, 128, 256, 512, 1024})
      if (bps == 0 || (unsigned long long)bps * 256 <= pairs) cands.push_back({3, h->cfg.threads, bps});
  const VqeConfig saved = h->cfg;
  double best = 1e300;
  VqeConfig best_cfg = saved;
  hipStream_t user = h->user_stream;
  h->user_stream = h->stream;
  for (const Cand& c : cands) {
    if (rc) break;
    rc = nwq_vqe_set_config(h, c.mode, c.threads, c.bps);
    if (rc) break;
    rc = eval_common(h, B, theta, nullptr, E, with_grad ? grad : nullptr, false);   // warm-up (and graph capture)
    if (rc) break;
    rc = check_hip(hipEventRecord(t0, h->stream), "hipEventRecord");
    for (int r = 0; r < 3 && !rc; ++r) rc = eval_common(h, B, theta, nullptr, E, with_grad ? grad : nullptr, false);
    if (!rc) rc = check_hip(hipEventRecord(t1, h->stream), "hipEventRecord");
    if (!rc) rc = check_hip(hipEventSynchronize(t1), "hipEventSynchronize");
    float ms = 0.f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
    if (!rc && ms / 3.0 < best) {
      best = ms / 3.0;
      best_cfg = h->cfg;
    }
  }
  h->user_stream = user;
  if (!rc) rc = nwq_vqe_set_config(h, best_cfg.mode, best_cfg.threads, best_cfg.blocks_per_state);
  else (void)nwq_vqe_set_config(h, saved.mode, saved.threads, saved.blocks_per_state);
  (void)hipStreamSynchronize(h->stream);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  for (void* p : {(void*)theta, (void*)E, (void*)grad})
    if (p) (void)hipFree(p);
  if (!rc && best_ms) *best_ms = best;
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One-call batched VQE for the Ising model (Sec. III, Fig. 4): the
// hardware-efficient ansatz and the open-chain transverse-field Ising
// Hamiltonian are built here, and the evaluation runs through a context kept
// per (device, n, L).  When (J, h) change, the context's term table is
// rewritten in place on the context's stream (the captured graphs read it at
// run time), so a new field costs no re-capture.
namespace {

struct BatchEntry {
  int device = -1, n = 0, L = 0;
  double J = 0.0, hx = 0.0;
  nwq_vqe_handle ctx = nullptr;
  std::vector<nwq::VqeTerm> terms;   // host copy of the table last uploaded (source of the async copy)
  unsigned long long used = 0;
};
constexpr size_t kBatchCacheMax = 8;
std::mutex g_batch_mu;
std::vector<BatchEntry> g_batch;
unsigned long long g_batch_clock = 0;

void tfim_terms(int n, double J, double hx, std::vector<nwq::VqeTerm>& out) {
  out.clear();
  for (int i = 0; i + 1 < n; ++i)
    out.push_back(nwq::VqeTerm{0ull, (1ull << i) | (1ull << (i + 1)), -J, 0, 0});
  for (int i = 0; i < n; ++i) out.push_back(nwq::VqeTerm{1ull << i, 0ull, -hx, 0, 0});
}

int batch_context(int device, int n, int L, double J, double hx, void* stream, BatchEntry** out) {
  for (auto& e : g_batch)
    if (e.device == device && e.n == n && e.L == L) {
      *out = &e;
      return NWQ_OK;
    }
  // ansatz: per layer RY on 0..n-1, RZ on 0..n-1, CX(0,1) .. CX(n-2,n-1)
  std::vector<int> types, qubits, params;
  for (int l = 0; l < L; ++l) {
    for (int axis = 0; axis < 2; ++axis)
      for (int q = 0; q < n; ++q) {
        types.push_back(axis == 0 ? NWQ_GATE_RY : NWQ_GATE_RZ);
        qubits.push_back(q);
        qubits.push_back(-1);
        params.push_back(l * 2 * n + axis * n + q);
      }
    for (int q = 0; q + 1 < n; ++q) {
      types.push_back(NWQ_GATE_CX);
      qubits.push_back(q);
      qubits.push_back(q + 1);
      params.push_back(-1);
    }
  }
  std::vector<nwq::VqeTerm> t;
  tfim_terms(n, J, hx, t);
  std::vector<uint64_t> xm, zm;
  std::vector<double> co;
  for (const auto& v : t) {
    xm.push_back(v.x);
    zm.push_back(v.z);
    co.push_back(v.c);
  }
  if (g_batch.size() >= kBatchCacheMax) {   // evict the least recently used context
    auto lru = std::min_element(g_batch.begin(), g_batch.end(),
                                [](const BatchEntry& a, const BatchEntry& b) { return a.used < b.used; });
    (void)nwq_vqe_destroy(lru->ctx);
    g_batch.erase(lru);
  }
  BatchEntry e;
  e.device = device;
  e.n = n;
  e.L = L;
  e.J = J;
  e.hx = hx;
  e.terms = t;
  int rc = nwq_vqe_create(n, (int)types.size(), types.data(), qubits.data(), params.data(), 2 * n * L, (int)t.size(),
                          xm.data(), zm.data(), co.data(), stream, &e.ctx);
  if (rc) return rc;
  g_batch.push_back(std::move(e));
  *out = &g_batch.back();
  return NWQ_OK;
}

}  // namespace

extern "C" {

int nwq_vqe_batch(int n, int L, const double* J_h, int B, const double* theta_dev, double* E_dev, double* grad_dev,
                  void* stream) {
  if (n < 1 || n > 30) return vqe_fail(NWQ_ERANGE, "nwq_vqe_batch needs 1..30 qubits");
  if (L < 1 || 2LL * n * L > (1LL << 24)) return vqe_fail(NWQ_EINVAL, "layer count out of range");
  if (!J_h || !std::isfinite(J_h[0]) || !std::isfinite(J_h[1])) return vqe_fail(NWQ_EINVAL, "J_h must hold finite J and h");
  if (B < 1 || B > 65535) return vqe_fail(NWQ_EINVAL, "batch size must be in [1, 65535]");
  if (!theta_dev || !E_dev) return vqe_fail(NWQ_EINVAL, "NULL theta or energy pointer");
  int device = 0;
  int rc = check_hip(hipGetDevice(&device), "hipGetDevice");
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(g_batch_mu);
  BatchEntry* e = nullptr;
  rc = batch_context(device, n, L, J_h[0], J_h[1], stream, &e);
  if (rc) return rc;
  e->used = ++g_batch_clock;
  nwq_vqe_handle h = e->ctx;
  h->user_stream = static_cast<hipStream_t>(stream);
  if (e->J != J_h[0] || e->hx != J_h[1]) {
    // rewrite the term table on the context's stream, after its earlier
    // evaluations; the host copy is reused, so the previous upload from it
    // must have finished
    rc = check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize(vqe batch)");
    e->J = J_h[0];
    e->hx = J_h[1];
    tfim_terms(n, e->J, e->hx, e->terms);
    h->terms = e->terms;
    if (!rc)
      rc = check_hip(hipMemcpyAsync(h->d_terms, e->terms.data(), e->terms.size() * sizeof(nwq::VqeTerm),
                                    hipMemcpyHostToDevice, h->stream), "hipMemcpyAsync(vqe terms)");
    if (rc) return rc;
  }
  return eval_common(h, B, theta_dev, nullptr, E_dev, grad_dev, false);
}

int nwq_vqe_batch_release(void) {
  std::lock_guard<std::mutex> lock(g_batch_mu);
  int rc = NWQ_OK;
  for (auto& e : g_batch) {
    const int r = nwq_vqe_destroy(e.ctx);
    if (r && !rc) rc = r;
  }
  g_batch.clear();
  return rc;
}

}  // extern "C"
