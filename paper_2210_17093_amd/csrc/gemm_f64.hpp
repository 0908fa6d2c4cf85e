// FP64 matrix-core GEMM for gfx950 (CDNA4), the contraction engine of every
// dense step of the qsGW iteration (AO->MO transform, Casida build, residues,
// qsGW self-energy matrix, Fock exchange).
//
//   C[b][m][n] = sum_{k in split z} A_b(m, k) * B_b(n, k)
//
// A and B are "operands": functors that return element (r, k) of a logical
// R x K matrix of batch b, with a compile-time flag telling whether k or r is
// the unit-stride direction (so global loads are coalesced either way).  The
// epilogue is a functor that receives each finished element.
//
// Tiling: BM x BN block tile, BK = 16 by default, 256 threads = 4 wave64 in a 2 x 2
// arrangement; each wave owns a (BM/2) x (BN/2) sub-tile made of 16 x 16
// accumulators updated by v_mfma_f64_16x16x4_f64.  Operands are staged in
// LDS in their global orientation ([r][k] for k-contiguous, [k][r] for
// r-contiguous, odd pitches), double buffered with one barrier per k-tile,
// and the next k-tile is prefetched into registers while the current one
// feeds the matrix cores.
//
// MFMA f64 16x16x4 lane layout (wave64):
//   A fragment: lane l holds A[l % 16][l / 16]      (16 rows x 4 k)
//   B fragment: lane l holds B[l / 16][l % 16]      (4 k x 16 cols)
//   D:          lane l, element q holds D[4 q + l / 16][l % 16]  (rows interleaved
//               across the four lane groups; measured on gfx950)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace qsgw {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Matrix-core instruction per compute type.  Both take the same 16 x 4 / 4 x 16
// operand fragments (lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]) and
// produce a 16 x 16 tile as four values per lane; `row` gives the tile row of
// value q of lane l (column l % 16).
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // f64 16x16x4 on gfx950: rows interleaved across the four lane groups
  __device__ __forceinline__ static int row(int lane, int q) { return 4 * q + (lane >> 4); }
};
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ __forceinline__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

// Split-BF16 products: each FP32 operand x is split as x = hi + lo with
// hi = bf16(x) and lo = bf16(x - hi) (both round to nearest even), and
// a*b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation.  The dropped lo_a lo_b and the rounding of lo leave a
// relative error of about 2^-16 per product; the three BF16 products run at
// several times the FP32 matrix-core rate.  Fragments: lane l holds the 8
// consecutive k = 8 (l / 16) .. 8 (l / 16) + 7 of row l % 16 of A (column
// l % 16 of B); D as in the FP32 16x16x4 instruction.
struct Bf16x3 {};
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
template <>
struct Mfma<Bf16x3> {
  typedef f32x4 acc_t;
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ __forceinline__ static acc_t mma(bf16x8 a, bf16x8 b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};
template <class T>
struct is_bf16x3 {
  static constexpr bool value = false;
};
template <>
struct is_bf16x3<Bf16x3> {
  static constexpr bool value = true;
};

// hi and lo halves of two split values (see Bf16x3), each pair packed in one
// 32-bit word (element 0 in the low half): two packed conversions, and hi is
// widened back to FP32 by placing its bits in the upper half of a word.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf16x2(float x0, float x1, uint32_t& hi, uint32_t& lo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x0, x1}, bf16x2));
  const float h0 = __builtin_bit_cast(float, hi << 16);
  const float h1 = __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x0 - h0, x1 - h1}, bf16x2));
}

// Split-BF16 LDS tiles are [r][k] with unpadded rows of BK values; the
// 16-byte chunk c (8 k) of row r sits at chunk c ^ x3_swizzle(r).  The
// swizzle spreads 8 consecutive rows of one chunk (a 16-byte access of 8
// lanes) over distinct 32-bank groups, and 16 consecutive rows over distinct
// 64-bank groups; two consecutive rows of one row run also share no bank.
__device__ __forceinline__ constexpr int x3_swizzle(int r) { return ((r >> 1) + (r >> 3)) & 3; }
template <int BK>
__device__ __forceinline__ constexpr int x3_at(int r, int k) {
  return r * BK + ((((k >> 3) ^ x3_swizzle(r)) << 3) | (k & 7));
}

// Element (r, k) at p[b*sb + r*sr + k*sk] (strides in elements of the
// storage type S, double or float); rows >= `rows` or k >= K read 0.
// Strided operands take the branch-free tile loader of the kernel: one base
// pointer per thread, a uniform stride between the thread's elements, and on
// edge tiles loads from a clamped (always valid) address followed by a select.
template <bool KC, class S = double>
struct Strided {
  static constexpr bool kContig = KC;
  static constexpr bool kStrided = true;
  typedef S storage_t;
  const S* p;
  int64_t sr, sk, sb;
  int64_t rows;
  __device__ __forceinline__ double get(int64_t b, int64_t r, int64_t k) const {
    return r < rows ? (double)p[b * sb + r * sr + k * sk] : 0.0;
  }
};

// Operands without the fast path (index arithmetic per element) leave
// kStrided false.
template <class OP, class = void>
struct is_strided_op {
  static constexpr bool value = false;
};
template <class OP>
struct is_strided_op<OP, decltype((void)OP::kStrided, void())> {
  static constexpr bool value = OP::kStrided;
};

// Rows that are pairs (m, k) of a symmetric N x N index, blocked in 2-D:
// row tile t covers the PM x PK block (blocks[t] = mb << 16 | kb) of pairs
// m = PM mb + i / PK, k = PK kb + i % PK, i = 0..PM*PK-1.  Element (row, kk)
// sits at p[b*sb + kk*sk + m*N + k].  Only blocks holding some m <= k are
// listed, so a symmetric product in (m, k) runs about half the pair space.
// Storage type S: double, or float for a rounded copy.
template <int PM, int PK, class S = double>
struct PairRows {
  static constexpr bool kContig = false;
  static constexpr bool kPairRows = true;
  static constexpr int kPM = PM, kPK = PK;
  typedef S storage_t;
  const S* p;
  int64_t sk, sb;
  int64_t n;              // N, the range of m and k
  const int32_t* blocks;  // one entry per row tile
};

template <class OP, class = void>
struct is_pair_rows_op {
  static constexpr bool value = false;
};
template <class OP>
struct is_pair_rows_op<OP, decltype((void)OP::kPairRows, void())> {
  static constexpr bool value = OP::kPairRows;
};

// Operand already split into BF16 halves (the split-BF16 products only), in
// k-blocks of 8: the 16-byte chunk (r, kb) of plane q (0 = hi, 1 = lo) holds
// k = 8 kb .. 8 kb + 7 of row r at p + q * ps + (kb * cs + r) * 8 (elements).
// Every tile is full: the producer pads K to a multiple of the k tile and
// the rows to cs >= the rows the launch covers, with zeros.
struct Split8 {
  static constexpr bool kContig = true;
  static constexpr bool kSplit8 = true;
  typedef uint32_t storage_t;  // registers hold the chunks' 32-bit words
  const uint16_t* p;
  int64_t cs;  // rows of a k-block slab
  int64_t ps;  // plane stride (elements)
  int64_t sb;  // batch stride (elements)
};

template <class OP, class = void>
struct is_split8_op {
  static constexpr bool value = false;
};
template <class OP>
struct is_split8_op<OP, decltype((void)OP::kSplit8, void())> {
  static constexpr bool value = OP::kSplit8;
};

// Chunks of a BR x BK split tile held by one of the 256 threads: chunk c is
// number q = c * 256 + tid, row q % BR, then (k-block, plane) from q / BR,
// k-block fastest.  With 256 / BR <= BK / 8 the plane is uniform per c.
template <int BR, int BK>
struct ChunkMap {
  static constexpr int C = BR * BK / 1024;  // chunks per thread (two planes)
  static constexpr int NKB = BK / 8;
  static_assert(256 % BR == 0 && 256 / BR <= NKB, "split tile shape");
  __device__ static constexpr int r(int tid) { return tid % BR; }
  __device__ static constexpr int kb(int tid, int c) { return (c * (256 / BR) + tid / BR) % NKB; }
  __device__ static constexpr int plane(int c) { return (c * (256 / BR)) / NKB; }
};

// Register type of an operand's prefetched elements: its storage type for
// strided and pair-row operands (float copies stay float), double otherwise.
template <class OP, class = void>
struct reg_type {
  typedef double type;
};
template <class OP>
struct reg_type<OP, decltype((void)sizeof(typename OP::storage_t), void())> {
  typedef typename OP::storage_t type;
};

// Pair (m, k) of row i of pair-row tile t (blocks as in PairRows).
template <int PM, int PK>
__device__ __forceinline__ void pair_of(const int32_t* blocks, int64_t t, int i, int64_t& m,
                                        int64_t& k) {
  const int32_t bk = blocks[t];
  m = (int64_t)(bk >> 16) * PM + i / PK;
  k = (int64_t)(bk & 0xffff) * PK + i % PK;
}

// Which elements of a BR x BK operand tile each of the 256 threads holds.
// Element e of thread tid sits at row rl(tid) + dr(e), k kl(tid) + dk(e): a
// per-thread origin plus a uniform step, so a thread addresses all its
// elements from one 32-bit offset.  Consecutive lanes read consecutive
// addresses in both orientations.
//   KB = false (FP64 / FP32 products, one element per lane and k step):
//     k-contiguous:  r = e*(256/BK) + tid/BK,  k = tid % BK
//     r-contiguous:  r = tid % BR,             k = e*(256/BR) + tid/BR
//   KB = true (split-BF16 products, whose fragments hold 8 consecutive k):
//     k-contiguous:  r = (e/4)*(1024/BK) + tid/(BK/4),  k = 4 (tid % (BK/4)) + e % 4
//     r-contiguous:  r = tid % BR,                      k = E (tid / BR) + e
template <int BR, int BK, bool KC, bool KB>
struct TileMap {
  static constexpr int E = BR * BK / 256;
  static constexpr int TK = BK / 4;  // KB, k-contiguous: threads along k
  __host__ __device__ static constexpr int rl(int tid) {
    return KC ? (KB ? tid / TK : tid / BK) : tid % BR;
  }
  __host__ __device__ static constexpr int kl(int tid) {
    return KC ? (KB ? 4 * (tid % TK) : tid % BK) : (KB ? E * (tid / BR) : tid / BR);
  }
  __host__ __device__ static constexpr int dr(int e) {
    return KC ? (KB ? (e / 4) * (256 / TK) : e * (256 / BK)) : 0;
  }
  __host__ __device__ static constexpr int dk(int e) {
    return KC ? (KB ? e % 4 : 0) : (KB ? e : e * (256 / BR));
  }
};

// Epilogues with a pass<ROWS, BN>(r0, n0, Cs, ldc, tid) member that takes one
// staged pass of the tile at a time.
template <class E, class = void>
struct has_pass_hook {
  static constexpr bool value = false;
};
template <class E>
struct has_pass_hook<E, decltype((void)E::kPassHook, void())> {
  static constexpr bool value = E::kPassHook;
};
// Pass epilogues of symmetric products (TRI): they receive every staged pass
// of an upper tile (diagonal tiles included) and drop the m > n elements and
// write the mirror themselves.
template <class E, class = void>
struct has_tri_pass {
  static constexpr bool value = false;
};
template <class E>
struct has_tri_pass<E, decltype((void)E::kTriPass, void())> {
  static constexpr bool value = E::kTriPass;
};

// Offset of element (r, k) of a split-BF16 LDS plane with br rows: swizzled
// [r][k] rows, or k-block-major [k/8][r][8] (KBM).
template <bool KBM, int BK>
__device__ __forceinline__ int x3_off(int br, int r, int k) {
  if constexpr (KBM)
    return ((k >> 3) * br + r) * 8 + (k & 7);
  else
    return x3_at<BK>(r, k);
}

// Element map of a split-BF16 operand tile, as a tag for the LDS store.
template <int BR, int BK, bool KC>
struct X3Map {
  typedef TileMap<BR, BK, KC, true> M;
  static constexpr int E = M::E;
  static constexpr bool kc = KC;
};

// Load this thread's E = BR*BK/256 elements of a BR x BK operand tile (rows
// r0.., k = kbase..) into v[], in the order of TileMap.
// `keep` returns whether this thread's elements are kept (false: they are
// zeros and the caller stores 0): full pair-row tiles load unconditionally
// and leave the masking to the LDS store, so that the loads of a tile are all
// in flight together instead of each waiting for its own select.
// Split-BF16 element map (KB = true): no element is zeroed here.  Loads of
// rows outside the operand read a clamped, valid element (their products only
// reach output rows the epilogue drops); k beyond the end of the range is
// clamped the same way and zeroed by the LDS store of the last k tile.
template <int BR, int BK, class OP, class R>
__device__ __forceinline__ void load_tile_kb(const OP& op, int64_t b, int64_t r0, int64_t kbase,
                                             int64_t kend, int tid, R* v) {
  typedef TileMap<BR, BK, OP::kContig, true> TM;
  constexpr int E = TM::E;
  const int rl = TM::rl(tid);
  const int kl = TM::kl(tid);
  const bool kfull = kbase + BK <= kend;
  const int kv = kfull ? BK : (int)(kend - kbase);  // valid k of the tile (uniform)
  if constexpr (is_split8_op<OP>::value) {
    typedef ChunkMap<BR, BK> CM;
    const uint16_t* origin = op.p + b * op.sb + ((kbase >> 3) * op.cs + r0) * 8;
#pragma unroll
    for (int c = 0; c < CM::C; ++c) {
      const char* sb = reinterpret_cast<const char*>(origin + CM::plane(c) * op.ps);
      const uint32_t off = (uint32_t)(((int64_t)CM::kb(tid, c) * op.cs + CM::r(tid)) * 16);
      const uint4 x = *reinterpret_cast<const uint4*>(sb + off);
      v[4 * c] = x.x;
      v[4 * c + 1] = x.y;
      v[4 * c + 2] = x.z;
      v[4 * c + 3] = x.w;
    }
  } else if constexpr (is_pair_rows_op<OP>::value) {
    static_assert(OP::kPM * OP::kPK == BR && 256 % BR == 0, "pair block must fill the row tile");
    typedef typename OP::storage_t S;
    int64_t m, k;
    pair_of<OP::kPM, OP::kPK>(op.blocks, r0 / BR, rl, m, k);
    const bool rok = (m < op.n) && (k < op.n);
    // a lane outside the pair range reads element (0, 0) of its k slab
    const uint32_t pofs = rok ? (uint32_t)((m * op.n + k) * (int64_t)sizeof(S)) : 0u;
    const S* origin = op.p + b * op.sb + kbase * op.sk;
    if (kfull) {
      const uint32_t toff = (uint32_t)((int64_t)kl * op.sk * (int64_t)sizeof(S)) + pofs;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const char* sb = reinterpret_cast<const char*>(origin + TM::dk(e) * op.sk);
        v[e] = (R)*reinterpret_cast<const S*>(sb + toff);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int kk = kl + TM::dk(e);
        const int kc = kk < kv ? kk : kv - 1;
        const char* sb = reinterpret_cast<const char*>(origin + (int64_t)kc * op.sk);
        v[e] = (R)*reinterpret_cast<const S*>(sb + pofs);
      }
    }
  } else if constexpr (is_strided_op<OP>::value) {
    static_assert(OP::kContig ? (256 % (BK / 4) == 0) : (256 % BR == 0),
                  "tile shape must divide the block");
    typedef typename OP::storage_t S;
    const S* origin = op.p + b * op.sb + r0 * op.sr + kbase * op.sk;
    const bool full = kfull && (r0 + BR <= op.rows);
    const uint32_t toff = (uint32_t)(((int64_t)rl * op.sr + (int64_t)kl * op.sk) * (int64_t)sizeof(S));
    if constexpr (OP::kContig && sizeof(S) == 4 && sizeof(R) == 4) {
      // Unit-stride FP32 rows whose 4-element runs are 16-byte aligned (uniform
      // test): one 16-byte load per run of 4 k, a wave covering whole rows.
      const bool vec = full && op.sk == 1 && (op.sr & 3) == 0 && (op.sb & 3) == 0 &&
                       (reinterpret_cast<uintptr_t>(op.p) & 15) == 0 && (kbase & 3) == 0;
      if (vec) {
#pragma unroll
        for (int g = 0; g < E / 4; ++g) {
          const char* sb = reinterpret_cast<const char*>(origin + TM::dr(4 * g) * op.sr);
          const f32x4 x = *reinterpret_cast<const f32x4*>(sb + toff);
          v[4 * g] = x[0];
          v[4 * g + 1] = x[1];
          v[4 * g + 2] = x[2];
          v[4 * g + 3] = x[3];
        }
        return;
      }
    }
    if (full) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const char* sb = reinterpret_cast<const char*>(origin + TM::dr(e) * op.sr + TM::dk(e) * op.sk);
        v[e] = (R)*reinterpret_cast<const S*>(sb + toff);
      }
    } else {
      const int rv = (r0 + BR <= op.rows) ? BR : (int)(op.rows - r0);  // valid rows (uniform)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = rl + TM::dr(e), kk = kl + TM::dk(e);
        const int rc = r < rv ? r : rv - 1, kc = kk < kv ? kk : kv - 1;
        v[e] = (R)origin[(int64_t)rc * op.sr + (int64_t)kc * op.sk];
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kk = kl + TM::dk(e);
      const int r = rl + TM::dr(e);
      v[e] = (R)op.get(b, r0 + r, kbase + (kk < kv ? kk : kv - 1));
    }
  }
}

template <int BR, int BK, class OP, class R>
__device__ __forceinline__ void load_tile_std(const OP& op, int64_t b, int64_t r0, int64_t kbase,
                                              int64_t kend, int tid, R* v, bool& keep) {
  constexpr bool KB = false;
  typedef TileMap<BR, BK, OP::kContig, KB> TM;
  constexpr int E = TM::E;
  keep = true;
  if constexpr (is_pair_rows_op<OP>::value) {
    static_assert(OP::kPM * OP::kPK == BR && 256 % BR == 0, "pair block must fill the row tile");
    // rows are unit-stride within a block row: thread owns one row i = tid % BR
    const int i = TM::rl(tid);
    const int kl = TM::kl(tid);
    int64_t m, k;
    pair_of<OP::kPM, OP::kPK>(op.blocks, r0 / BR, i, m, k);
    const bool rok = (m < op.n) && (k < op.n);
    typedef typename OP::storage_t S;
    const bool kfull = kbase + BK <= kend;
    const S* origin = op.p + b * op.sb + kbase * op.sk;
    const uint32_t pofs = rok ? (uint32_t)((m * op.n + k) * (int64_t)sizeof(S)) : 0u;
    if (kfull) {
      // Full k tile: one uniform base per element (scalar registers) and one
      // 32-bit per-lane offset; a lane outside the pair range reads element
      // (0, 0) of its k slab, which exists, and discards it.
      const uint32_t toff = (uint32_t)((int64_t)kl * op.sk * (int64_t)sizeof(S)) + pofs;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const char* sb = reinterpret_cast<const char*>(origin + TM::dk(e) * op.sk);
        v[e] = (R)*reinterpret_cast<const S*>(sb + toff);
      }
      keep = rok;
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t kk = kl + TM::dk(e);
        const bool ok = rok && kbase + kk < kend;
        const char* sb = reinterpret_cast<const char*>(ok ? origin + kk * op.sk : op.p);
        const S x = *reinterpret_cast<const S*>(sb + (ok ? pofs : 0u));
        v[e] = ok ? (R)x : (R)0;
      }
    }
  } else if constexpr (is_strided_op<OP>::value) {
    static_assert(OP::kContig ? (256 % (KB ? BK / 4 : BK) == 0) : (256 % BR == 0),
                  "tile shape must divide the block");
    // Uniform part (scalar registers): the tile origin and the element step.
    // Per-thread part: one 32-bit byte offset shared by all E elements.
    const int rl = TM::rl(tid);
    const int kl = TM::kl(tid);
    typedef typename OP::storage_t S;
    const S* origin = op.p + b * op.sb + r0 * op.sr + kbase * op.sk;
    const uint32_t toff = (uint32_t)(((int64_t)rl * op.sr + (int64_t)kl * op.sk) * (int64_t)sizeof(S));
    const bool full = (r0 + BR <= op.rows) && (kbase + BK <= kend);
    if (full) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const char* sb = reinterpret_cast<const char*>(origin + TM::dr(e) * op.sr + TM::dk(e) * op.sk);
        v[e] = (R)*reinterpret_cast<const S*>(sb + toff);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = rl + TM::dr(e);
        const int k = kl + TM::dk(e);
        const bool ok = (r0 + r < op.rows) && (kbase + k < kend);
        // masked elements read the tile origin, which is always a valid element
        const char* sb = reinterpret_cast<const char*>(
            ok ? origin + TM::dr(e) * op.sr + TM::dk(e) * op.sk : origin);
        const S x = *reinterpret_cast<const S*>(sb + (ok ? toff : 0u));
        v[e] = ok ? (R)x : (R)0;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kk = TM::kl(tid) + TM::dk(e);
      const int r = TM::rl(tid) + TM::dr(e);
      const int64_t k = kbase + kk;
      v[e] = (k < kend) ? (R)op.get(b, r0 + r, k) : (R)0;
    }
  }
}

template <int BR, int BK, bool KB, class OP, class R>
__device__ __forceinline__ void load_tile(const OP& op, int64_t b, int64_t r0, int64_t kbase,
                                          int64_t kend, int tid, R* v, bool& keep) {
  if constexpr (KB) {
    keep = true;
    load_tile_kb<BR, BK>(op, b, r0, kbase, kend, tid, v);
  } else {
    load_tile_std<BR, BK>(op, b, r0, kbase, kend, tid, v, keep);
  }
}

// Host check: the tile loaders address a thread's elements with one 32-bit
// byte offset from a uniform origin; it must fit for the operand's strides
// (BR rows x BK k per tile, 256 threads, element map KB).
template <class OP>
inline bool loader_offsets_fit(const OP& op, int BR, int BK = 16, bool KB = false) {
  const uint64_t E = (uint64_t)BR * BK / 256;
  if constexpr (is_split8_op<OP>::value) {
    return KB && ((uint64_t)(BK / 8 - 1) * (uint64_t)op.cs + BR) * 16 < (1ull << 32);
  } else if constexpr (is_pair_rows_op<OP>::value) {
    // pair offset plus the lane's k offset
    const uint64_t kl = KB ? BK - E : 256 / BR - 1;
    return ((uint64_t)op.n * (uint64_t)op.n + kl * (uint64_t)op.sk) *
               sizeof(typename OP::storage_t) < (1ull << 32);
  } else if constexpr (is_strided_op<OP>::value) {
    uint64_t rl, kl;
    if (OP::kContig) {
      rl = KB ? 1024 / BK - 1 : 256 / BK - 1;
      kl = KB ? BK - 4 : BK - 1;
    } else {
      rl = BR - 1;
      kl = KB ? BK - E : 256 / BR - 1;
    }
    return (rl * (uint64_t)op.sr + kl * (uint64_t)op.sk) * sizeof(typename OP::storage_t) <
           (1ull << 32);
  } else {
    return true;
  }
}

// Hardware dispatches consecutive workgroup ids round-robin over the 8 XCDs
// (each with its own L2).  Renumber so that each XCD walks a contiguous range
// of logical tiles: neighbouring tiles share operand panels in one L2.
__device__ __forceinline__ int64_t xcd_logical_id(int64_t bid, int64_t nwg) {
  constexpr int64_t NXCD = 8;
  if (nwg < NXCD) return bid;
  const int64_t xcd = bid % NXCD, local = bid / NXCD;
  const int64_t q = nwg / NXCD, r = nwg % NXCD;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

struct TileCoord {
  int64_t tm, tn;
};

// Grouped ordering: GROUP_M row tiles sweep all column tiles before the next
// group starts, bounding the live A and B panels.
__device__ __forceinline__ TileCoord grouped_tile(int64_t id, int64_t tiles_m, int64_t tiles_n) {
  constexpr int64_t GROUP_M = 8;
  const int64_t per_group = GROUP_M * tiles_n;
  const int64_t g = id / per_group;
  const int64_t first_m = g * GROUP_M;
  const int64_t gsz = (tiles_m - first_m) < GROUP_M ? (tiles_m - first_m) : GROUP_M;
  const int64_t in = id - g * per_group;
  return {first_m + in % gsz, in / gsz};
}

// Upper-triangular tile pairs tm <= tn, numbered column by column:
// id = tn (tn + 1) / 2 + tm.
__device__ __forceinline__ TileCoord tri_tile(int64_t id) {
  int64_t tn = (int64_t)((sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
  while (tn * (tn + 1) / 2 > id) --tn;
  while ((tn + 1) * (tn + 2) / 2 <= id) ++tn;
  return {id - tn * (tn + 1) / 2, tn};
}

// Row-tile map: the launch enumerates `tiles_m` row tiles, and the map turns
// that index into the row tile actually computed.  The identity covers the
// whole output; a table skips row tiles whose outputs are all unneeded
// without leaving idle workgroups in the launch (idle workgroups would also
// unbalance the per-XCD work, as each XCD owns a contiguous range).
struct AllTiles {
  __device__ __forceinline__ int64_t operator()(int64_t t) const { return t; }
};


// TRI: only tiles with tm <= tn run, elements with m > n are dropped and the
// epilogue is asked to mirror (m, n) -> (n, m) (symmetric results).
// T: double or float (v_mfma_*_16x16x4), or Bf16x3 (split-BF16 products).
template <int BM, int BN, class OA, class OB, class EPI, bool TRI, class FILT, int BK, class T>
__device__ __forceinline__ void gemm_body(const OA& A, const OB& B, const EPI& epi, int64_t M,
                                          int64_t N, int64_t K, int64_t kchunk, int64_t tiles_m,
                                          int64_t tiles_n, int64_t nbatch, const FILT& filt,
                                          int64_t lid) {
  constexpr bool X3 = is_bf16x3<T>::value;
  static_assert(BK % (X3 ? 32 : 4) == 0, "BK is a multiple of the MFMA depth");
  // LDS layout per operand.  FP64 / FP32: a k-contiguous operand is kept
  // [r][k] (pitch BK+1) so global rows land in LDS rows without a transpose;
  // an r-contiguous one is kept [k][r] (pitch BR+1).  Both pitches are odd,
  // which keeps the 16 lanes of an MFMA fragment read on distinct banks.
  // Split-BF16: hi and lo tiles, both [r][k] whatever the global orientation
  // (a fragment is 8 consecutive k of one row, one 16-byte read), in the
  // chunk-swizzled layout of x3_at.
  constexpr bool AK = OA::kContig, BKC = OB::kContig;
  constexpr int SZA = X3 ? BM * BK : (AK ? BM * (BK + 1) : BK * (BM + 1));
  constexpr int SZB = X3 ? BN * BK : (BKC ? BN * (BK + 1) : BK * (BN + 1));
  constexpr int EA = BM * BK / 256;
  constexpr int EB = BN * BK / 256;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(BM % 32 == 0 && BN % 32 == 0, "tile must split into 2x2 waves of 16x16 MFMA tiles");
  static_assert(EA >= 1 && EB >= 1, "tile too small for 256 threads");
  static_assert(!X3 || ((AK || EA % 8 == 0) && (BKC || EB % 8 == 0)),
                "split-BF16 r-contiguous tiles store 8 consecutive k per thread");
  typedef typename std::conditional<X3, __bf16, T>::type LT;  // LDS element type
  constexpr int NPL = X3 ? 2 : 1;                               // planes (hi, lo)

  // One LDS block: the double-buffered operand tiles during the K loop, then
  // the FP64 staging area of the epilogue (WM rows of the C tile at a time).
  constexpr int LDC = BN + 1;
  constexpr size_t OPER_BYTES = 2 * NPL * (size_t)(SZA + SZB) * sizeof(LT);
  constexpr size_t STAGE_BYTES = (size_t)WM * LDC * sizeof(double);
  constexpr size_t SMEM_BYTES = OPER_BYTES > STAGE_BYTES ? OPER_BYTES : STAGE_BYTES;
  __shared__ __attribute__((aligned(16))) char smem[SMEM_BYTES];
  // plane p of buffer u: As[u * NPL + p]
  LT (*As)[SZA] = reinterpret_cast<LT (*)[SZA]>(smem);
  LT (*Bs)[SZB] = reinterpret_cast<LT (*)[SZB]>(smem + 2 * NPL * (size_t)SZA * sizeof(LT));
  typedef Mfma<T> MM;
  // element (r, k) of the staged FP64 / FP32 tiles
  auto a_at = [](int r, int k) { return AK ? r * (BK + 1) + k : k * (BM + 1) + r; };
  auto b_at = [](int r, int k) { return BKC ? r * (BK + 1) + k : k * (BN + 1) + r; };

  // The launch is one-dimensional over (split, batch, tile), tile fastest.
  // Workgroups go to the XCDs round-robin by this linear id; renumbering
  // gives each XCD a contiguous logical range, so the tiles that share one
  // K chunk (or one batch entry) share one L2.
  const int64_t ntiles = TRI ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
  const int64_t id = lid % ntiles;
  const int64_t rest = lid / ntiles;
  const int64_t batch = rest % nbatch;
  const int64_t split = rest / nbatch;
  TileCoord tc = TRI ? tri_tile(id) : grouped_tile(id, tiles_m, tiles_n);
  const int64_t m0 = (TRI ? tc.tm : filt(tc.tm)) * BM, n0 = tc.tn * BN;
  if (m0 >= M || n0 >= N) return;
  const int64_t kb0 = split * kchunk;
  const int64_t kb1 = (kb0 + kchunk) < K ? (kb0 + kchunk) : K;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * WM;
  const int wn = (wave & 1) * WN;

  typename MM::acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = MM::zero();

  typename reg_type<OA>::type ra[EA];
  typename reg_type<OB>::type rb[EB];
  bool keep_a = true, keep_b = true;
  int kv_next = BK;  // split-BF16: valid k of the k tile held in the prefetch registers

  auto gload = [&](int64_t kbase) {
    load_tile<BM, BK, X3>(A, batch, m0, kbase, kb1, tid, ra, keep_a);
    load_tile<BN, BK, X3>(B, batch, n0, kbase, kb1, tid, rb, keep_b);
    if constexpr (X3) kv_next = kbase + BK <= kb1 ? BK : (int)(kb1 - kbase);
  };
  // Split-BF16 store of one operand's elements (TileMap<.., KB = true>
  // order): runs of consecutive k of one row go out as 16-byte (r-contiguous:
  // 8 k) or 8-byte (k-contiguous: 4 k) writes to the hi and lo planes.  In
  // the last, partial k tile (kv < BK valid k, uniform) the k beyond the range
  // are stored as zeros.
  // Pre-split operands: each chunk goes to its plane as one 16-byte write.
  auto sstore_split = [&](const uint32_t* v, LT* hi, LT* lo, auto map_tag) {
    typedef decltype(map_tag) CM;
#pragma unroll
    for (int c = 0; c < CM::C; ++c) {
      LT* dst = CM::plane(c) ? lo : hi;
      *reinterpret_cast<uint4*>(dst + x3_at<BK>(CM::r(tid), 8 * CM::kb(tid, c))) =
          uint4{v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]};
    }
  };
  auto sstore_x3 = [&](auto* v, int kv, LT* hi, LT* lo, auto map_tag) {
    typedef decltype(map_tag) MP;
    constexpr int E = MP::E;
    constexpr int RUN = MP::kc ? 4 : 8;
    if (kv < BK) {
      // (the empty asm makes the bound opaque, so that the compares stay in
      // this rarely taken branch instead of being hoisted into every k tile;
      // kv is uniform over the workgroup, readfirstlane puts it in a scalar
      // register also where the compiler could not prove that)
      int kvo = __builtin_amdgcn_readfirstlane(kv);
      asm volatile("" : "+s"(kvo));
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (MP::M::kl(tid) + MP::M::dk(e) >= kvo) v[e] = 0;
    }
#pragma unroll
    for (int g = 0; g < E / RUN; ++g) {
      const int r = MP::M::rl(tid) + MP::M::dr(g * RUN);
      const int k = MP::M::kl(tid) + MP::M::dk(g * RUN);
      uint32_t h[RUN / 2], l[RUN / 2];
#pragma unroll
      for (int u = 0; u < RUN / 2; ++u)
        split_bf16x2((float)v[g * RUN + 2 * u], (float)v[g * RUN + 2 * u + 1], h[u], l[u]);
      const int o = x3_at<BK>(r, k);
      if constexpr (RUN == 8) {
        *reinterpret_cast<uint4*>(hi + o) = uint4{h[0], h[1], h[2], h[3]};
        *reinterpret_cast<uint4*>(lo + o) = uint4{l[0], l[1], l[2], l[3]};
      } else {
        *reinterpret_cast<uint2*>(hi + o) = uint2{h[0], h[1]};
        *reinterpret_cast<uint2*>(lo + o) = uint2{l[0], l[1]};
      }
    }
  };
  auto sstore = [&](int buf) {
    if constexpr (X3) {
      if constexpr (is_split8_op<OA>::value)
        sstore_split(ra, As[2 * buf], As[2 * buf + 1], ChunkMap<BM, BK>());
      else
        sstore_x3(ra, kv_next, As[2 * buf], As[2 * buf + 1], X3Map<BM, BK, AK>());
      if constexpr (is_split8_op<OB>::value)
        sstore_split(rb, Bs[2 * buf], Bs[2 * buf + 1], ChunkMap<BN, BK>());
      else
        sstore_x3(rb, kv_next, Bs[2 * buf], Bs[2 * buf + 1], X3Map<BN, BK, BKC>());
    } else {
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const int idx = e * 256 + tid;
        const int kk = OA::kContig ? (idx % BK) : (idx / BM);
        const int r = OA::kContig ? (idx / BK) : (idx % BM);
        As[buf][a_at(r, kk)] = keep_a ? (T)ra[e] : (T)0;
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int idx = e * 256 + tid;
        const int kk = OB::kContig ? (idx % BK) : (idx / BN);
        const int r = OB::kContig ? (idx / BK) : (idx % BN);
        Bs[buf][b_at(r, kk)] = keep_b ? (T)rb[e] : (T)0;
      }
    }
  };

  // Split-BF16 products of one staged k tile (buffer cur).  KBM: tiles held
  // k-block-major ([k/8][r][8] per plane, as direct-to-LDS loads write them)
  // instead of the swizzled [r][k] rows.
  auto mma_x3 = [&](int cur, auto kbm_tag) {
    if constexpr (X3) {
    constexpr bool KBM = decltype(kbm_tag)::value;
    auto at = [&](int br, int r, int k) { return x3_off<KBM, BK>(br, r, k); };
    const LT* ah_s = As[2 * cur];
    const LT* al_s = As[2 * cur + 1];
    const LT* bh_s = Bs[2 * cur];
    const LT* bl_s = Bs[2 * cur + 1];
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
      const int kofs = ks * 32 + 8 * (lane >> 4);
      bf16x8 bh[TN], bl[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = at(BN, wn + j * 16 + (lane & 15), kofs);
        bh[j] = *reinterpret_cast<const bf16x8*>(bh_s + o);
        bl[j] = *reinterpret_cast<const bf16x8*>(bl_s + o);
      }
      // one row block of A at a time (fewer live fragments); the TN
      // accumulators of a row block interleave, so consecutive products
      // never wait on each other: small cross terms first, then hi * hi
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int o = at(BM, wm + i * 16 + (lane & 15), kofs);
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(ah_s + o);
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(al_s + o);
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MM::mma(al, bh[j], acc[i][j]);
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MM::mma(ah, bl[j], acc[i][j]);
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MM::mma(ah, bh[j], acc[i][j]);
      }
    }
    }
  };

  const int64_t nk = kb1 > kb0 ? (kb1 - kb0 + BK - 1) / BK : 0;
  if constexpr (X3 && is_split8_op<OA>::value && is_split8_op<OB>::value) {
    // Both operands pre-split (every tile full): the chunks go from global
    // memory straight into LDS (global_load_lds_dwordx4: each lane's 16 bytes
    // land at the wave's LDS base + 16 x lane), one k tile ahead, in the
    // k-block-major layout that a wave's 64 consecutive rows of one k-block
    // and plane fill contiguously.
    typedef __attribute__((address_space(3))) void lds_void;
    typedef __attribute__((address_space(1))) void glob_void;
    auto issue = [&](const auto& op, int64_t r0, int64_t kbase, LT* hi, LT* lo, auto br_tag) {
      constexpr int BR = decltype(br_tag)::value;
      typedef ChunkMap<BR, BK> CM;
      const uint16_t* origin = op.p + batch * op.sb + ((kbase >> 3) * op.cs + r0) * 8;
#pragma unroll
      for (int c = 0; c < CM::C; ++c) {
        const int q0 = c * 256 + wave * 64;  // chunk of lane 0: rows r_w .. r_w + 63
        const int rw = q0 % BR, rest = q0 / BR;
        const int kb = rest % CM::NKB, pl = rest / CM::NKB;
        const uint16_t* src = origin + pl * op.ps + ((int64_t)kb * op.cs + rw + lane) * 8;
        LT* dst = (pl ? lo : hi) + (kb * BR + rw) * 8;
        __builtin_amdgcn_global_load_lds((glob_void*)src, (lds_void*)dst, 16, 0, 0);
      }
    };
    auto issue_tile = [&](int64_t kbase, int buf) {
      issue(A, m0, kbase, As[2 * buf], As[2 * buf + 1], std::integral_constant<int, BM>());
      issue(B, n0, kbase, Bs[2 * buf], Bs[2 * buf + 1], std::integral_constant<int, BN>());
    };
    if (nk > 0) {
      issue_tile(kb0, 0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
    for (int64_t it = 0; it < nk; ++it) {
      const int cur = (int)(it & 1);
      // (the other buffer's tile was consumed before the previous barrier)
      if (it + 1 < nk) issue_tile(kb0 + (it + 1) * BK, cur ^ 1);
      mma_x3(cur, std::true_type());
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
  } else {
    if (nk > 0) {
      gload(kb0);
      sstore(0);
      __syncthreads();
    }
    for (int64_t it = 0; it < nk; ++it) {
      const int cur = (int)(it & 1);
      if (it + 1 < nk) gload(kb0 + (it + 1) * BK);
      if constexpr (X3) {
        mma_x3(cur, std::false_type());
      } else {
        const T* as = As[cur];
        const T* bs = Bs[cur];
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
          const int krow = ks * 4 + (lane >> 4);
          T a[TM], b[TN];
#pragma unroll
          for (int i = 0; i < TM; ++i) a[i] = as[a_at(wm + i * 16 + (lane & 15), krow)];
#pragma unroll
          for (int j = 0; j < TN; ++j) b[j] = bs[b_at(wn + j * 16 + (lane & 15), krow)];
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
              acc[i][j] = MM::mma(a[i], b[j], acc[i][j]);
        }
      }
      if (it + 1 < nk) sstore(cur ^ 1);
      __syncthreads();
    }
  }

  // Epilogue through LDS, one wave-row (WM rows of the tile) per pass: the
  // two waves owning those rows store their accumulators straight from the
  // matrix-core registers, then all 256 threads apply the epilogue row by row
  // (consecutive threads on consecutive columns).  Keeping the arithmetic out
  // of the accumulator registers stops the compiler from copying all of them
  // to VGPRs at once, which would halve the occupancy of the K loop.
  if (nk > 0) __syncthreads();  // operand buffers are free once every wave is done
  if constexpr (has_pass_hook<EPI>::value && X3) {
    // FP32 accumulators: the whole tile is staged at once as FP32 (the size of
    // half the tile in FP64) and handed to the epilogue in one pass
    static_assert(!TRI, "pass epilogues of full tiles");
    static_assert((size_t)BM * LDC * sizeof(float) <= SMEM_BYTES, "FP32 staging fits");
    float* Cf = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          Cf[(wm + i * 16 + MM::row(lane, q)) * LDC + wn + j * 16 + (lane & 15)] = acc[i][j][q];
    __syncthreads();
    epi.template pass<BM, BN>(m0, n0, Cf, LDC, tid);
    __syncthreads();  // (a persistent caller reuses the LDS for its next tile)
  } else {
  double* Cs = reinterpret_cast<double*>(smem);
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    if ((wave >> 1) == pass) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            Cs[(i * 16 + MM::row(lane, q)) * LDC + wn + j * 16 + (lane & 15)] = (double)acc[i][j][q];
    }
    __syncthreads();
    if constexpr (has_pass_hook<EPI>::value) {
      // epilogues that take a whole staged pass (rows m0 + pass WM .., all
      // columns of the tile; they check their own ranges)
      static_assert(!TRI || has_tri_pass<EPI>::value,
                    "pass epilogues of full tiles, or ones that handle the triangle");
      epi.template pass<WM, BN>(m0 + pass * WM, n0, Cs, LDC, tid);
    } else {
      for (int idx = tid; idx < WM * BN; idx += 256) {
        const int row = idx / BN, col = idx - (idx / BN) * BN;
        const int64_t m = m0 + pass * WM + row;
        const int64_t n = n0 + col;
        if (m < M && n < N) {
          const double v = Cs[row * LDC + col];
          if (TRI) {
            if (m <= n) epi(batch, split, m, n, v, m != n);
          } else {
            epi(batch, split, m, n, v, false);
          }
        }
      }
    }
    __syncthreads();
  }
  }
}

// Single problem: the launch is one-dimensional over (split, batch, tile).
template <int BM, int BN, class OA, class OB, class EPI, bool TRI, class FILT = AllTiles,
          int BK = 16, class T = double>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(OA A, OB B, EPI epi, int64_t M, int64_t N,
                                                       int64_t K, int64_t kchunk, int64_t tiles_m,
                                                       int64_t tiles_n, int64_t nbatch, FILT filt) {
  const int64_t lid = xcd_logical_id((int64_t)blockIdx.x, (int64_t)gridDim.x);
  gemm_body<BM, BN, OA, OB, EPI, TRI, FILT, BK, T>(A, B, epi, M, N, K, kchunk, tiles_m, tiles_n,
                                                   nbatch, filt, lid);
}

// One job of a grouped launch: a whole problem of the single-problem kernel
// (its own operands, epilogue, sizes, split plan), owning the workgroups
// [wg_begin, wg_begin + tiles * nbatch * nsplit) of the launch.
template <class OA, class OB, class EPI>
struct GemmJob {
  OA a;
  OB b;
  EPI e;
  int64_t M, N, K, kchunk, tiles_m, tiles_n, nbatch;
  int64_t wg_begin;
};

// Grouped launch: many independent problems of different sizes (one per
// molecule of a batch) in one dispatch.  The `total` workgroup tiles of all
// jobs are split into gridDim.x contiguous ranges, one per workgroup (one
// tile each when the grid covers them all; a persistent grid of a few
// workgroups per compute unit walks longer ranges).  Each tile finds its job
// by binary search over the jobs' first tile ids, then runs the same tile
// body as the single-problem kernel.
template <int BM, int BN, class OA, class OB, class EPI, bool TRI, int BK = 16, class T = double>
__global__ __launch_bounds__(256, 2) void gemm_grouped_kernel(const GemmJob<OA, OB, EPI>* jobs,
                                                              int64_t njobs, int64_t total) {
  const int64_t lid = xcd_logical_id((int64_t)blockIdx.x, (int64_t)gridDim.x);
  const int64_t G = gridDim.x;
  const int64_t t0 = lid * total / G, t1 = (lid + 1) * total / G;
  for (int64_t g = t0; g < t1; ++g) {
    int64_t lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (jobs[mid].wg_begin <= g) lo = mid; else hi = mid - 1;
    }
    const GemmJob<OA, OB, EPI>& j = jobs[lo];
    gemm_body<BM, BN, OA, OB, EPI, TRI, AllTiles, BK, T>(j.a, j.b, j.e, j.M, j.N, j.K, j.kchunk,
                                                         j.tiles_m, j.tiles_n, j.nbatch, AllTiles(),
                                                         g - j.wg_begin);
  }
}

// ---------------------------------------------------------------- epilogues
// C[b or z][m][n] = alpha * v  (mirror writes (n, m) too)
struct EpiStore {
  double* c;
  int64_t ldc;
  int64_t sb;       // stride per batch index
  int64_t sz;       // stride per split index (partial sums)
  double alpha;
  float* c32 = nullptr;  // optional FP32 copy, same layout (not with split-K)
  bool nt = false;  // non-temporal stores: large outputs read by a later kernel, whole lines
                    // (partly written lines of a non-temporal store reach HBM unmerged)
  __device__ __forceinline__ void put(double* p, double x) const {
    if (nt)
      __builtin_nontemporal_store(x, p);
    else
      *p = x;
  }
  __device__ __forceinline__ void put(float* p, float x) const {
    if (nt)
      __builtin_nontemporal_store(x, p);
    else
      *p = x;
  }
  __device__ __forceinline__ void operator()(int64_t b, int64_t z, int64_t m, int64_t n, double v,
                                             bool mirror) const {
    double* cb = c + b * sb + z * sz;
    const double x = alpha * v;
    put(&cb[m * ldc + n], x);
    if (mirror) put(&cb[n * ldc + m], x);
    if (c32) {
      float* fb = c32 + b * sb;
      put(&fb[m * ldc + n], (float)x);
      if (mirror) put(&fb[n * ldc + m], (float)x);
    }
  }
};

}  // namespace qsgw
