// Internal declarations shared by the engine's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nwq.h"

namespace nwq {

using cd = std::complex<double>;

constexpr int kBlock = 256;          // threads per workgroup for streaming kernels
constexpr int kWave = 64;            // CDNA wavefront width

// Gate / superoperator matrices passed by value as kernel arguments.
struct Mat2 { double2 m[4]; };       // 2x2, row-major
struct Mat4 { double2 m[16]; };      // 4x4, row-major
struct Diag4 { double2 d[4]; };      // diagonal entries indexed by u = b0 + 2 b1

// Qubit set of a k-qubit dense kernel (k <= 4).
struct QSet {
  int sorted[4];                     // ascending positions (zero-insertion order)
  unsigned long long off[4];         // 2^{q_j} in the operator's own order
};

// Streaming launch shape chosen by the autotuner (per kernel class and
// target bucket).
struct LaunchCfg {
  int ppt = 4;                       // pairs / groups / elements per thread (1, 2, 4, 8; 16 where allowed;
                                     // 32, 64, 128: split-workgroup kernels of 256, 512, 1024 threads)
  int nt = 0;                        // flags: bit 0 non-temporal loads and stores; bit 1 (shapes 32, 64,
                                     // 128 only) XCD-contiguous workgroup order
};

// Launch shapes are kept in three buckets per class, by the lowest target
// bit of the launch: below 3 the partner amplitudes of a group share one
// 128-byte line (a non-temporal hint then costs a second fetch of the line);
// from 3 to 10 the streams of a group are within 16 KiB of each other; from
// 11 up they are 32 KiB or more apart.  The best shape differs between them
// (on MI355X at 30 qubits: 1 group per thread, 16 with the hint, 4 with the
// hint for the 2x2 kernel).
constexpr int kBuckets = 3;
constexpr int kMaxTargetBits = 64;   // lowest target bits with their own tuned launch shape
inline int bucket_of(int lowest_bit) { return lowest_bit < 3 ? 0 : (lowest_bit < 11 ? 1 : 2); }

// Kernel classes (also the timing classes of nwq_timing_read).
enum KClass {
  KC_RESET = 0, KC_SV1Q = 1, KC_DIAG = 2, KC_PERM = 3, KC_SV2Q = 4,
  KC_FUSED = 5, KC_DM1 = 6, KC_DM2 = 7, KC_REDUCE = 8, KC_COUNT = 9
};

// ---- launchers (kernels_sv.hip) -------------------------------------------
void launch_fill_basis0(hipStream_t s, double2* a, unsigned long long len);
void launch_sv_1q(hipStream_t s, double2* a, int nbits, int q, const Mat2& m, const LaunchCfg& cfg);
void launch_sv_diag(hipStream_t s, double2* a, int nbits, int q0, int q1, const Diag4& d, const LaunchCfg& cfg);
void launch_sv_swap1(hipStream_t s, double2* a, int nbits, int q, const LaunchCfg& cfg);
void launch_sv_swap2(hipStream_t s, double2* a, int nbits, int qa, int qb,
                     unsigned long long offA, unsigned long long offB, const LaunchCfg& cfg);
void launch_sv_2q(hipStream_t s, double2* a, int nbits, int q0, int q1, const Mat4& m, const LaunchCfg& cfg);
// k-qubit operator on the given qubits (operator index bit j = qubits[j]);
// dev_matrix is the dense 2^k x 2^k, or with pauli (k = 4 only) the 32-entry
// compact form of a Pauli-pattern 16 x 16: the 16 diagonal entries, then the
// 4 x 4 among operator indices 0, 5, 10, 15.
void launch_sv_kq(hipStream_t s, double2* a, int nbits, int k, const int* qubits, const double2* dev_matrix,
                  const LaunchCfg& cfg, bool pauli = false);

// ---- reductions (kernels_reduce.hip) --------------------------------------
// One pass of the tiled Pauli-term kernel.  `terms` is a device table of
// `count` TermDev rows; partial sums go to partials[row * grid + block] with
// row = first_row + term index.
struct TermDev {
  unsigned long long xl;    // x mask in tile-local bit positions
  unsigned long long zl;    // z bits inside the tile, tile-local positions
  unsigned long long zo;    // z bits outside the tile, global positions
  int y;                    // popcount(x & z) mod 4
  int pad;
};
struct TileShape {
  int c;                    // low contiguous bits in the tile
  int m;                    // number of high bits
  int hi[8];                // the high bit positions, ascending
};
int pauli_tile_grid(int nbits, const TileShape& t);
// Terms with no flipped bits (x = 0): up to 16 z masks (global bit
// positions) by value; partials as above, with the same grid.
struct ZMasks {
  unsigned long long z[16];
};
void launch_pauli_diag(hipStream_t s, const double2* a, int nbits, const ZMasks& zs, int count, double* partials,
                       int first_row, int grid);
void launch_pauli_tile(hipStream_t s, const double2* a, int nbits, const TileShape& t,
                       const TermDev* terms, int count, double* partials, int first_row, int grid);
// One term with wide x support, pairs read from global memory; partials[block].
void launch_pauli_pairs(hipStream_t s, const double2* a, int nbits, unsigned long long x, unsigned long long z,
                        int y, double* partials, int grid);
// DM: Tr(rho P_t) for each term, complex partials partials[(2*row + {0,1}) * grid + block].
int dm_pauli_grid(int n);
void launch_dm_pauli(hipStream_t s, const double2* rho, int n, const TermDev* terms, int count,
                     double* partials, int grid);
// sum |a_j|^2 over len entries into partials[block]
int sumsq_grid(unsigned long long len);
void launch_sumsq(hipStream_t s, const double2* a, unsigned long long len, double* partials, int grid);
// out[r] = sum_b partials[r * grid + b] (fixed order); if coeffs: out[rows] = sum_r coeffs[r] out[r]
void launch_reduce_rows(hipStream_t s, const double* partials, int rows, int grid,
                        const double* coeffs, double* out);

// ---- fused LDS blocks (kernels_fuse.hip) ----------------------------------
struct FusedOp {            // one gate inside a fused block, tile-local bits
  int kind;                 // 0: 1q dense, 1: 1q diag, 2: 2q dense, 3: 2q member swap, 4: 2q diag,
                            // 6: 1q diag read from a 2x2 entry (M[0], M[3]; register-blocked kernels only),
                            // 7: dense 16x16 over all four register bits, in register order (4-bit kernel),
                            // 8: the same with the pattern of a Pauli channel after a diagonal gate: diagonal
                            //    except for a dense 4x4 among register indices 0, 5, 10, 15 (4-bit kernel)
  int lo, hi;               // sorted tile-local bit positions (hi unused for 1q)
  int o0, o1;               // kind 2: local offsets of q0, q1; kind 3: offsets swapped; kind 4: local bits of q0, q1
  int mat;                  // start of its matrix in the block program's matrix table (double2 units)
  int code;                 // register-blocked kernels: rb_op_code() of the fields above
  int real00;               // kind 0: 1 when M[0][0] is real (U3, RX), 2 when all of M is (RY, H);
                            // the imaginary parts known to be zero are skipped
};
// One switch index per register-blocked op (kind and register bits): 0 + B
// dense 2x2, 4 + B diagonal (M[0], M[1]), 8 + B diagonal (M[0], M[3]); with
// u = 4 o0 + o1: 16 + u dense 4x4, 32 + u CX, 48 + u SWAP, 64 + u 2q diagonal;
// 84 + B dense 2x2 with a real M[0][0], 88 + B real dense 2x2; 96 dense 16x16
// over the four register bits, 97 its Pauli-channel pattern (the 16 diagonal
// entries, then the 4x4 among registers 0, 5, 10, 15; 4-register-bit kernel
// only).
constexpr int kRbCodeCopy = 80;   // kernel-internal copy that pads an odd gate count
constexpr int kRbCodeDense16 = 96;
constexpr int kRbCodePauli16 = 97;
inline int rb_op_code(const FusedOp& op) {
  const int u = 4 * op.o0 + op.o1;
  switch (op.kind) {
    case 0: return op.real00 == 2 ? 88 + op.lo : (op.real00 == 1 ? 84 + op.lo : op.lo);
    case 1: return 4 + op.lo;
    case 6: return 8 + op.lo;
    case 7: return kRbCodeDense16;
    case 8: return kRbCodePauli16;
    case 2: return 16 + u;
    case 3: return 32 + u;
    case 5: return 48 + u;
    default: return 64 + u;   // 4
  }
}
struct FusedBlockDev {
  int c, m;                 // tile = low c bits + m high bits
  int hi[8];
  int op_begin, op_count;   // range in the op table
  // register-blocked kernels: global offset of tile entry j * 2^(k - rbits)
  // (the per-thread part of an entry's index is added to it)
  unsigned long long joff[16];
  // Register-blocked SV kernel: bit 0 = the first phase's register bits all
  // lie above the low c tile bits, so its registers are loaded straight from
  // HBM (register j from the tile entry at jdir[j] plus the thread's part);
  // bit 1 = the same for the last phase, stored straight to HBM (sdir).
  // Such a phase skips its LDS round trip and barrier.
  int direct;
  unsigned long long jdir[16], sdir[16];
};
void launch_fused_block(hipStream_t s, double2* a, int nbits, const FusedBlockDev& blk,
                        const FusedOp* ops, const double2* mats, int lds_k);
// Register-blocked blocks: blk.op_begin / op_count index a phase table; each
// phase holds rbits (3 or 4) register bits (tile-local, ascending; unused
// entries of reg ignored) and a range of ops whose lo / o0 / o1 fields are
// register-bit indices below rbits.  Tiles of 2^k amplitudes, 8 <= k <= 13,
// 2^(k-rbits) threads.  Op kinds as FusedOp plus 5 = SWAP (o0, o1).
struct FusedPhase {
  int reg[4];
  int op_begin, op_count;
  int pad0, pad1;
  // Register-blocked SV kernel: the padded LDS offset (over the phase's
  // register bits) that register j is loaded from and stored to.  Permutation
  // gates at the start or the end of a phase are folded into these.
  unsigned short ld_off[16], st_off[16];
};
// ld_perm[j] / st_perm[j]: register-bit index whose entry register j loads /
// stores (nullptr: identity); offsets padded by one entry per 16.
inline void fill_phase_offsets(FusedPhase& fp, int rbits, const int* ld_perm, const int* st_perm) {
  auto off = [&](int p) {
    unsigned o = 0;
    for (int r = 0; r < rbits; ++r)
      if ((p >> r) & 1) o |= 1u << fp.reg[r];
    return (unsigned short)(o + (o >> 4));
  };
  for (int j = 0; j < 16; ++j) {
    const bool in = j < (1 << rbits);
    fp.ld_off[j] = in ? off(ld_perm ? ld_perm[j] : j) : 0;
    fp.st_off[j] = in ? off(st_perm ? st_perm[j] : j) : 0;
  }
}
size_t fused_rb_lds_bytes(int k);
// enable_dynamic_lds for every register-blocked instance (outside graph capture)
int fused_rb_enable_lds();
// batch > 1: blockIdx.y = batch element b works on a + b * 2^nbits with the
// matrix table mats + b * mat_stride; max_grid caps the tiles' grid (0 = 2^20).
// flags: kFusedNonTemporal = non-temporal global loads and stores of the
// tiles; kFusedDirect = load the first phase / store the last phase straight
// between HBM and registers where the block allows it (FusedBlockDev::direct).
// max_tiles > 0 runs only the first max_tiles tiles of each state, and
// tile_mask != ~0 only the tiles whose index is zero outside tile_mask (the
// block leaves the others alone: used when they are known to hold zeros,
// which a block maps to zeros).
constexpr int kFusedNonTemporal = 1;
constexpr int kFusedDirect = 2;
// SV circuits (host side): gate products before the blocks are planned, where
// they save FP64 work (circuit.hip, gate_products).
constexpr int kFusedGateFusion = 4;
void launch_fused_rb(hipStream_t s, double2* a, int nbits, const FusedBlockDev& blk, const FusedPhase* phases,
                     const FusedOp* ops, const double2* mats, int rbits, int batch = 1, int mat_stride = 0,
                     int max_grid = 0, int flags = 0, unsigned long long max_tiles = 0,
                     unsigned long long tile_mask = ~0ull);

// ---- error handling (engine.hip) ------------------------------------------
int set_error(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// Dynamic LDS above 64 KiB: up to the CU's whole 160 KiB less the kernel's
// static LDS (the LDS-resident VQE kernel takes up to that; the fused tiles at
// most 2^13 amplitudes plus one padding entry per 16).  enable_dynamic_lds
// raises a kernel's limit to it once per kernel and device, under a lock: the
// limit is process-wide state of the kernel, so setting it per launch from
// several host threads raced with launches of the same kernel elsewhere, and a
// smaller value set for one launch could undercut another's.
constexpr int kMaxDynamicLds = 160 * 1024;
int enable_dynamic_lds(const void* kernel);

}  // namespace nwq
