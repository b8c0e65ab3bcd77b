// Learned position model: a 16 -> 64 -> 64 -> 1 MLP on MFMA that predicts an
// address's elementary-interval index, a per-segment error bound that turns
// the prediction into a bounded exact search, and the hand-written training
// kernels (forward, backward, Adam).  This is an addition to the paper's
// method; exactness never depends on the model: every window search is
// verified, and a failed check falls back to the tree descent of Section 3.
//
// Matrix layout.  Every product is v_mfma_f32_16x16x16bf16_1k on one
// wavefront with the hidden units as rows and 16 addresses as columns
// (A: row l%16, k = 4(l/16)+i; B: k = 4(l/16)+i, column l%16; C: row
// 4(l/16)+i, column l%16).  Computing the transposed activations makes each
// layer's C registers the next layer's B operand without any data movement.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "burst_tiles.hpp"
#include "descent.hpp"
#include "learned.hpp"

namespace planb {

constexpr int kH = 64, kF = 16;
constexpr int oW1 = 0, ob1 = oW1 + kH * kF, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, ow3 = ob2 + kH, ob3 = ow3 + kH;
constexpr int kParams = ob3 + 1;  // 5313
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f2bf(float f)
{
    union {
        float f;
        uint32_t u;
    } cv{f};
    uint32_t u = cv.u;
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40);  // NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Per-lane MFMA A operands of the two weight matrices (40 VGPRs).
struct MlpRegs {
    s4 w1[4];     // W1[16mb + l%16][4g + i]
    s4 w2[4][4];  // W2[16mb + l%16][16kb + 4g + i]
};

__device__ inline void load_regs(const uint16_t* wb, MlpRegs& R)
{
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) R.w1[mb][i] = (short)wb[oW1 + (16 * mb + c) * kF + 4 * g + i];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) R.w2[mb][kb][i] = (short)wb[oW2 + (16 * mb + c) * kH + 16 * kb + 4 * g + i];
}

// B operand of layer 1: bytes 4g..4g+3 of the column's address, as bf16 of byte/256 (exact).
__device__ inline s4 feature_operand(uint64_t xhi, uint64_t xlo)
{
    const int g = (threadIdx.x & 63) >> 4;
    const uint64_t word = g < 2 ? xhi : xlo;
    const int sh = (g & 1) ? 24 : 56;
    s4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float f = (float)((word >> (sh - 8 * i)) & 0xFF) * (1.0f / 256.0f);
        v[i] = (short)(__float_as_uint(f) >> 16);
    }
    return v;
}

struct Activations {
    f4 h1[4];   // relu(layer 1), float32, C layout
    s4 h1b[4];  // the same rounded to bf16 (layer-2 B operand)
    f4 h2[4];   // relu(layer 2), float32, C layout
};

// Forward pass for the wavefront's 16 columns; lanes of one column must hold
// the same address.  Returns y for column l%16 (in all four lanes of it).
__device__ inline float mlp_forward(const MlpRegs& R, const float* sb1, const float* sb2, const float* sw3, float b3,
                                    uint64_t xhi, uint64_t xlo, Activations& A)
{
    const int g = (threadIdx.x & 63) >> 4;
    const s4 xb = feature_operand(xhi, xlo);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        f4 z = {0.f, 0.f, 0.f, 0.f};
        z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.w1[mb], xb, z, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float v = fmaxf(z[i] + sb1[16 * mb + 4 * g + i], 0.f);
            A.h1[mb][i] = v;
            A.h1b[mb][i] = (short)f2bf(v);
        }
    }
    float part = 0.f;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.w2[mb][kb], A.h1b[kb], z, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int u = 16 * mb + 4 * g + i;
            const float v = fmaxf(z[i] + sb2[u], 0.f);
            A.h2[mb][i] = v;
            part = fmaf(sw3[u], v, part);
        }
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    return part + b3;
}

// ---- inference forward pass (the lookups, the error table and
// planb_model_predict all use this one; training uses mlp_forward above).
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Weight operands of mlp_infer (40 VGPRs).  Layer 1 takes the address bytes
// as integers (0..255, exact in bf16) against W1 / 256: scaling by a power of
// two is exact, so every product equals W1 * byte/256.  Layer 2 runs as two
// v_mfma_f32_16x16x32_bf16 per row block: in chunk q of the 64 hidden units,
// lane group g's slots 0..3 and 4..7 hold units 32q + 4g + j and
// 32q + 16 + 4g + j, which are exactly its layer-1 C registers of row blocks
// 2q and 2q + 1; W2 is loaded in the same unit order, so the contraction is
// the same sum and nothing moves between the layers.
struct InferRegs {
    s4 w1[4];     // (W1 / 256)[16mb + l%16][4g + i]
    bf8 w2[4][2];  // W2[16mb + l%16][unit(q, g, j)]
};

__device__ inline __bf16 bf_bits(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// The per-row constants of mlp_infer held in registers (40 VGPRs): this
// lane's rows 16mb + 4g + i of b1 and b2 (the accumulators start from them)
// and of w3 (bf16, two per register).  Reading them from LDS for every tile
// made LDS bandwidth the limit of the whole forward pass.
struct InferConsts {
    f4 b1[4], b2[4];
    uint32_t w3[8];  // w3[16mb + 4g + 2k], w3[16mb + 4g + 2k + 1] as bf16 bits, low half first
};

// Both loaders read runs of 4 consecutive parameters with one 8- or 16-byte
// load (every offset below is a multiple of 4 parameters, and the parameter
// arrays are allocation-aligned): the multi-FIB kernel reloads them whenever
// a wavefront's tile changes table, so their cost is paid per 64 lookups.
__device__ inline void load_consts(const ModelDesc& M, InferConsts& C)
{
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const float4 v1 = *reinterpret_cast<const float4*>(M.w + ob1 + 16 * mb + 4 * g);
        const float4 v2 = *reinterpret_cast<const float4*>(M.w + ob2 + 16 * mb + 4 * g);
        C.b1[mb] = f4{v1.x, v1.y, v1.z, v1.w};
        C.b2[mb] = f4{v2.x, v2.y, v2.z, v2.w};
        // w3[16mb + 4g + 2k], w3[16mb + 4g + 2k + 1]: low half first, as stored
        const uint2 w3 = *reinterpret_cast<const uint2*>(M.wb + ow3 + 16 * mb + 4 * g);
        C.w3[2 * mb] = w3.x;
        C.w3[2 * mb + 1] = w3.y;
    }
}

__device__ inline void load_infer(const uint16_t* wb, InferRegs& R)
{
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const uint2 v = *reinterpret_cast<const uint2*>(wb + oW1 + (16 * mb + c) * kF + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t word = i < 2 ? v.x : v.y;
            const uint16_t bits = (uint16_t)((i & 1) ? word >> 16 : word & 0xFFFFu);
            const __bf16 w = (__bf16)(bf2f(bits) * (1.0f / 256.0f));
            R.w1[mb][i] = (short)__builtin_bit_cast(uint16_t, w);
        }
    }
    // K slots 0..3 of chunk q are units 32q + 4g + j, slots 4..7 units 32q + 16 + 4g + j
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint16_t* row = wb + oW2 + (16 * mb + c) * kH + 32 * q;
            const uint2 lo = *reinterpret_cast<const uint2*>(row + 4 * g);
            const uint2 hi = *reinterpret_cast<const uint2*>(row + 16 + 4 * g);
            typedef uint32_t u4 __attribute__((ext_vector_type(4)));
            R.w2[mb][q] = __builtin_bit_cast(bf8, u4{lo.x, lo.y, hi.x, hi.y});
        }
}

// ReLU on the bit pattern: one integer max.  A float whose sign bit is set
// (negative, or -0) is a negative integer, and non-negative floats order as
// their bit patterns do.
__device__ inline float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// y for the wavefront's 16 columns (address of column l%16 in every lane of
// that column).  Same arithmetic definition as mlp_forward: h1 rounded to bf16
// (round to nearest even, here by the hardware conversion), fp32 accumulation
// (the accumulators start from the biases).
__device__ inline float mlp_infer(const InferRegs& R, const InferConsts& C, float b3, uint64_t xhi, uint64_t xlo)
{
    const int g = (threadIdx.x & 63) >> 4;
    // bytes 4g .. 4g + 3 of the address, most significant first, as bf16 integers
    const uint32_t w = (uint32_t)((g < 2 ? xhi : xlo) >> ((g & 1) ? 0 : 32));
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    typedef float fl2 __attribute__((ext_vector_type(2)));
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    // two bytes per conversion instruction (exact: integers below 256)
    const bf2 b01 = __builtin_convertvector(fl2{(float)(w >> 24), (float)((w >> 16) & 0xFFu)}, bf2);
    const bf2 b23 = __builtin_convertvector(fl2{(float)((w >> 8) & 0xFFu), (float)(w & 0xFFu)}, bf2);
    const s4 xb = __builtin_bit_cast(s4, u2{__builtin_bit_cast(uint32_t, b01), __builtin_bit_cast(uint32_t, b23)});
    // h1 = bf16(ReLU(z)) = ReLU(bf16(z)) (rounding keeps the sign), so round two
    // values at a time and take the ReLU of the packed pair with one 16-bit max
    uint32_t hp[2][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const f4 z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.w1[mb], xb, C.b1[mb], 0, 0, 0);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            typedef short sh2 __attribute__((ext_vector_type(2)));
            const bf2 pr = __builtin_convertvector(fl2{z[2 * k], z[2 * k + 1]}, bf2);
            const sh2 v = __builtin_elementwise_max(__builtin_bit_cast(sh2, pr), sh2{0, 0});
            hp[mb >> 1][2 * (mb & 1) + k] = __builtin_bit_cast(uint32_t, v);
        }
    }
    bf8 h[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        h[q] = __builtin_bit_cast(bf8, u4{hp[q][0], hp[q][1], hp[q][2], hp[q][3]});
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        f4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R.w2[mb][0], h[0], C.b2[mb], 0, 0, 0);
        z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R.w2[mb][1], h[1], z, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t pair = C.w3[2 * mb + i / 2];
            const float w3 = __uint_as_float((i & 1) ? (pair & 0xFFFF0000u) : (pair << 16));
            acc[i] = fmaf(w3, relu_bits(z[i]), acc[i]);
        }
    }
    float part = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    return part + b3;
}

// Stage biases and w3 (as float) in LDS.
__device__ inline void stage_small(const ModelDesc& M, float* sb1, float* sb2, float* sw3)
{
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        sb1[i] = M.w[ob1 + i];
        sb2[i] = M.w[ob2 + i];
        sw3[i] = bf2f(M.wb[ow3 + i]);
    }
}

__device__ inline uint64_t predict_position(float y, uint64_t m)
{
    const float pm = y * (float)m;
    if (!(pm >= 1.0f)) return 0;  // negative, tiny or NaN
    if (pm >= (float)m) return m - 1;
    // m < 2^32 for a learned model, so 1 <= pm < (float)m <= 2^32 and the
    // floor fits 32 bits (a 32-bit conversion, not the 64-bit sequence)
    const uint64_t p = (uint32_t)floorf(pm);
    return p < m ? p : m - 1;
}

// The error table's segment of position p: floor(p * S / m), exactly (p < m <
// 2^32; inv_m = 1.0f / m), as the table is built.  While S <= 2^20 a float
// estimate is within one of the quotient (q < 2^20 and the estimate's
// relative error is a few 2^-24), and one exact 64-bit product corrects it;
// larger tables divide.
__device__ inline uint32_t segment_of(uint64_t p, uint32_t S, uint64_t m, float inv_m)
{
    const uint64_t a = p * (uint64_t)S;
    if (S > (1u << 20)) return (uint32_t)(a / m);
    uint64_t q = (uint64_t)((float)a * inv_m);
    const uint64_t qm = q * m;
    if (qm > a)
        --q;  // one too high
    else if (a - qm >= m)
        ++q;  // one too low
    return (uint32_t)q;
}

// A lookup's segment: the float estimate p * S / m, without the correction
// (within one of the exact segment, from 4 instructions instead of a 64-bit
// division of about 55).  An estimate off by one at a segment boundary reads
// the neighbouring segment's bound; if that window then misses x, the
// window's verification fails and the lookup falls back, so results stay
// exact.
__device__ inline uint32_t lookup_segment(uint64_t p, const ModelDesc& M)
{
    const uint32_t s = (uint32_t)((float)(uint32_t)p * M.seg_scale);  // p < m < 2^32: the same float
    return s < M.segments ? s : M.segments - 1;
}


// One-lane descent (every key of each node) of the subtree rooted at node
// `node` of level `level`: the interval of x, when it lies in that subtree.
template <int B, int KB>
__device__ inline uint64_t descend_from(const TreeDesc& t, uint32_t level, uint32_t node, uint64_t xhi, uint64_t xlo)
{
    using KF = KeyFmt<KB>;
    const auto* keys = static_cast<const typename KF::T*>(t.keys);
    uint32_t q = node;
    for (uint32_t l = level; l + 1 < t.depth; ++l) {
        const size_t nb = (size_t)(t.off[l] + q) * B;
        uint32_t c = 0;
#pragma unroll
        for (int s = 0; s < B; ++s) c += KF::le(keys[nb + s], xhi, xlo);
        q = min(q * B + c, t.last[l + 1]);
    }
    constexpr int LC = leaf_cap_for(B, (int)sizeof(typename KF::T)), LS = leaf_slots_for(B, (int)sizeof(typename KF::T));
    const size_t nb = t.leaf_base + (size_t)q * LS;
    uint32_t c = 0;
#pragma unroll
    for (int s = 0; s < LC; ++s) c += KF::le(keys[nb + leaf_key_slot(s, (int)sizeof(typename KF::T))], xhi, xlo);
    const uint64_t idx = (uint64_t)q * LC + c - 1;
    return idx < t.m_minus_1 ? idx : t.m_minus_1;
}

// The whole tree, one lane (fallbacks).
template <int B, int KB>
__device__ inline uint64_t descend_lane(const TreeDesc& t, uint64_t xhi, uint64_t xlo)
{
    return descend_from<B, KB>(t, 0, 0, xhi, xlo);
}

constexpr int kLearnBlock = 256;

// One wavefront step of the learned lookup: addresses [base, base + 64) of a
// batch of n (4 MFMA tiles of 16), then one lane per address for the window
// search, verification and fallback.  R and C hold the model's weight
// operands and per-row constants.
// Lookups whose window check fails: with QUEUE they are appended to a queue
// in scratch memory and searched afterwards by fallback_kernel, so that a
// wavefront never waits for one lane's whole-tree descent; without it (the
// multi-FIB kernel) the failing lanes descend the tree in place.
struct FallbackQueue {
    uint32_t* count;  // entries appended (zeroed before the lookup)
    uint32_t* idx;    // address index of each entry; cap entries
    uint32_t cap;     // >= the lookups of the launch
};

template <int B, int KB, bool QUEUE>
__device__ inline void learned_step(const TreeDesc& t, const ModelDesc& M, const InferRegs& R, const InferConsts& C,
                                    float b3, const u64x2* addrs, uint64_t base, uint64_t n, uint16_t* out,
                                    uint32_t* fallbacks, const FallbackQueue& fq)
{
    using KF = KeyFmt<KB>;
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    const uint64_t m = t.m_minus_1 + 1;
    float y = 0.f;
    uint64_t xhi = 0, xlo = 0;
#pragma unroll
    for (int tile = 0; tile < 4; ++tile) {
        const uint64_t i = base + 16 * tile + c;
        const u64x2 a = __builtin_nontemporal_load(addrs + (i < n ? i : n - 1));
        const float yt = mlp_infer(R, C, b3, a.x, a.y);
        if (g == tile) {
            y = yt;
            xhi = a.x;
            xlo = a.y;
        }
    }
    // this lane's address is base + 16g + c = base + l
    const uint64_t p = predict_position(y, m);
    const uint32_t seg = lookup_segment(p, M);
    const uint32_t e0 = M.eps[seg];
    // widen the bound by half plus 16: interior addresses can err a little
    // more than the sampled points; a wider window costs at most a level more.
    // An empty segment (no bound) takes the whole tree.
    const uint64_t e = e0 != kEmpty ? (uint64_t)e0 + (e0 >> 1) + 16 : m;
    const uint64_t lo = p > e ? p - e : 0, hi = p + e < m - 1 ? p + e : m - 1;
    // x's interval lies in the window [lo, hi] when the model is within its
    // bound, and then its leaf in the smallest subtree holding the leaves of lo
    // and hi: lane groups descend that subtree with whole-node reads (a few
    // levels) instead of one lane binary-searching the window key by key.  The
    // descent itself tells whether x lies in the subtree, so no key of the
    // window is read to check it: the separators it compared bound x from
    // below by the first key of the leaf it reached and from above by the
    // first key of the next leaf, except at the subtree's two ends.  So the
    // leaf's count of keys <= x is the exact interval unless it is 0 (x below
    // the subtree's first key) or counts every key of the subtree's last leaf
    // while another leaf follows (x may lie beyond it); those lookups fall back.
    constexpr uint32_t LC = (uint32_t)leaf_cap_for(B, (int)sizeof(typename KF::T));
    uint32_t a = (uint32_t)lo / LC, b = (uint32_t)hi / LC, level = t.depth - 1;  // lo <= hi < m < 2^32
    while (a != b) {
        a /= (uint32_t)B;
        b /= (uint32_t)B;
        --level;
    }
    // groups of G = 4 lanes take the wavefront's 64 subtrees in G rounds: round
    // u serves owner lane (u % G) * LPW + lane / G (the plain lookup's hand-off)
    using D = Descent<B, B / 4, 1, KB, false>;
    constexpr int G = D::G, LPW = D::LPW, T = G;
    const int grp = l / G, jg = l % G;
    uint64_t yh[T], yl[T];
    uint32_t pv[T], sl[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int owner = (u % G) * LPW + grp;
        yh[u] = D::shfl64(xhi, owner);
        yl[u] = KB == 16 ? D::shfl64(xlo, owner) : 0;
        pv[u] = (uint32_t)__shfl((int)a, owner, 64);
        sl[u] = (uint32_t)__shfl((int)level, owner, 64);
    }
    // bit u: round u's descent has taken the last child at every level so far,
    // so its leaf is the subtree's last (internal nodes are full except at the
    // tree's right edge, where no leaf follows)
    uint32_t rightmost = (1u << T) - 1u;
    const auto* gkeys = static_cast<const typename D::K*>(t.keys);
    for (uint32_t lv = 0; lv + 1 < t.depth; ++lv) {
        const uint32_t off = t.off[lv], lim = t.last[lv + 1];
#pragma unroll
        for (int u = 0; u < T; ++u)
            if (lv >= sl[u]) {  // the same for the group's G lanes
                const uint32_t c =
                    D::template node_count<false>(gkeys, (typename D::SlotIdx)(off + pv[u]) * B, jg, yh[u], yl[u]);
                rightmost &= c == (uint32_t)(B - 1) ? ~0u : ~(1u << u);
                pv[u] = min(pv[u] * B + c, lim);
            }
    }
    uint32_t res[T], cnt[T];
    if constexpr (D::kBlockLane) {
        D::template leaf_blocks<T>(t, gkeys, pv, yh, yl, jg, l - jg, 0, res, cnt);
    } else {
        uint32_t idx[T];
        uint16_t hop[T];
        D::template leaf_groups<T>(t, gkeys, pv, yh, yl, jg, l - jg, idx, hop, cnt);
#pragma unroll
        for (int u = 0; u < T; ++u) res[u] = hop[u];
    }
    // bit 16 of a result marks a lookup that falls back (hops are 16 bits)
    const uint32_t last_leaf = t.last[t.depth - 1];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const bool open_top = ((rightmost >> u) & 1u) && cnt[u] == LC && pv[u] < last_leaf;
        res[u] = (res[u] & 0xFFFFu) | (cnt[u] == 0 || open_top ? 0x10000u : 0u);
    }
    // this lane's own result: round r * G + lane / LPW, from group lane % LPW
    const int gsel = l / LPW, src = (l % LPW) * G;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const uint32_t got = (uint32_t)__shfl((int)res[k], src, 64);
        v = k == gsel ? got : v;
    }
    const bool ok = (v & 0x10000u) == 0;
    v &= 0xFFFFu;
    const uint64_t i = base + l;
    const bool need = !ok && i < n;
    if constexpr (QUEUE) {
        // one atomic per wavefront reserves the queue entries of its failing lanes
        const uint64_t mask = __ballot(need);
        if (mask) {
            const int first_lane = __builtin_ctzll(mask);
            uint32_t first = 0;
            if (l == first_lane) first = atomicAdd(fq.count, (uint32_t)__popcll(mask));
            first = (uint32_t)__builtin_amdgcn_readlane((int)first, first_lane);
            const uint32_t slot = first + (uint32_t)__popcll(mask & ((1ull << l) - 1ull));
            if (need && slot < fq.cap) fq.idx[slot] = (uint32_t)i;  // cap >= n: always taken
        }
        if (ok && i < n) __builtin_nontemporal_store((uint16_t)v, out + i);
    } else {
        if (need) v = t.vals[descend_lane<B, KB>(t, xhi, xlo)];
        if (i < n) __builtin_nontemporal_store((uint16_t)v, out + i);
        if (fallbacks) {
            const uint64_t mask = __ballot(need);
            if (l == 0 && mask) atomicAdd(fallbacks, (uint32_t)__popcll(mask));
        }
    }
}

// Learned lookup of one batch (grid stride over 64-address wavefront steps).
// QUEUE: failing lookups go to the queue fq; else each descends the tree in
// place and fq.count (when not null) counts them.
template <int B, int KB, bool QUEUE>
__global__ void __launch_bounds__(kLearnBlock)
learned_kernel(TreeDesc t, ModelDesc M, const u64x2* __restrict__ addrs, uint64_t n, uint16_t* __restrict__ out,
               FallbackQueue fq)
{
    InferRegs R;
    load_infer(M.wb, R);
    InferConsts C;
    load_consts(M, C);
    const float b3 = M.w[ob3];
    const uint64_t wave = (uint64_t)blockIdx.x * (kLearnBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kLearnBlock / 64);
    for (uint64_t base = wave * 64; base < n; base += nwaves * 64) {
        if constexpr (QUEUE)
            learned_step<B, KB, true>(t, M, R, C, b3, addrs, base, n, out, nullptr, fq);
        else
            learned_step<B, KB, false>(t, M, R, C, b3, addrs, base, n, out, fq.count, FallbackQueue{});
    }
}

// ---------------------------------------------------------------- learned lookup over leaf tops
// The learned lookup for trees with 64-bit key slots whose leaf minima fit in
// LDS.  Every leaf's first key is kept as its top 32 bits ("leaf tops", built
// once per FIB); each workgroup stages them, with the error table, in LDS.
// The model's window [p - w, p + w] of interval positions maps to a range of
// leaves; a binary search over that range of the tops (in LDS) finds the last
// leaf whose top is <= x's top half.  The window is verified on the tops
// themselves: the first leaf of the range must have a top <= x's, and the
// leaf after the range a top > x's.  A tie (the found leaf's top equals x's)
// is settled with whole keys, walking back over the tied leaves, exactly as
// the plain lookup settles the bottom internal level; the first such read is
// issued before the lane hand-off and used after it.  Then G = 4 lanes per
// lookup read the leaf (one line) and pick the answer as the plain lookup
// does.  A lookup whose window fails its check goes to the fallback queue.
struct LeafTops {
    const uint32_t* tops;  // top 32 bits of each leaf's first key
    uint32_t nleaves;
};

// LDS of learned_tops_kernel: the leaf tops, the error table, and 16 bytes
// for the workgroup's largest error bound.
__host__ __device__ inline size_t learned_tops_lds_bytes(uint32_t nleaves, uint32_t segments)
{
    return ((size_t)nleaves + 3) / 4 * 16 + ((size_t)segments + 3) / 4 * 16 + 16;
}

// QUEUE: failing lookups go to the queue fq; else each descends the tree in
// place and fq.count (when not null) counts them.
template <int B, int KPL, int R, int BS, bool QUEUE>
__global__ void __launch_bounds__(BS)
learned_tops_kernel(TreeDesc t, ModelDesc M, LeafTops lt, const u64x2* __restrict__ addrs, uint64_t n,
                    uint16_t* __restrict__ out, FallbackQueue fq)
{
    using D = Descent<B, KPL, R, 8, true>;
    static_assert(D::G == 4 && D::kBlockLane, "one 32-byte leaf block per lane");
    constexpr int G = D::G, LPW = D::LPW, T = R * G;
    constexpr uint32_t LC = (uint32_t)D::kLC;
    extern __shared__ uint4 lds_raw[];
    uint32_t* tops = reinterpret_cast<uint32_t*>(lds_raw);
    uint32_t* eps = tops + ((size_t)lt.nleaves + 3) / 4 * 4;
    uint32_t* emax_lds = eps + ((size_t)M.segments + 3) / 4 * 4;  // the largest bound (kEmpty if a segment is empty)
    if (threadIdx.x == 0) *emax_lds = 0;
    __syncthreads();
    stage_items<8>(
        lt.nleaves, threadIdx.x, BS, [&](uint32_t i) { return lt.tops[i]; }, [&](uint32_t i, uint32_t v) { tops[i] = v; });
    uint32_t emax = 0;
    stage_items<8>(
        M.segments, threadIdx.x, BS, [&](uint32_t i) { return M.eps[i]; },
        [&](uint32_t i, uint32_t e) {
            eps[i] = e;
            emax = max(emax, e);
        });
    if (emax) atomicMax(emax_lds, emax);
    __syncthreads();
    // Every window covers at most `span` leaves: its positions p - w .. p + w
    // (w = 2 e0 + 16 <= 2 emax + 16) fall in at most 2w / LC + 2 leaves, and an
    // empty segment's window is every leaf.  The window search below takes the
    // same power-of-two steps in every lane, from `top`, the largest power of
    // two <= span, down to 1; they reach any count up to 2 top - 1 >= span.
    uint32_t top;
    {
        const uint32_t em = *emax_lds;
        uint64_t span = lt.nleaves;
        if (em != kEmpty) span = min(span, 2 * (2 * (uint64_t)em + 16) / LC + 2);
        top = 1u << (31 - __builtin_clz((uint32_t)span));  // span >= 1
        top = (uint32_t)__builtin_amdgcn_readfirstlane((int)top);
    }
    InferRegs Rg;
    load_infer(M.wb, Rg);
    InferConsts C;
    load_consts(M, C);
    const float b3 = M.w[ob3];
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    const uint64_t m = t.m_minus_1 + 1;
    const uint32_t last_leaf = lt.nleaves - 1;
    const auto* gkeys = static_cast<const uint64_t*>(t.keys);
    const uint64_t wave = (uint64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (BS / 64);
    const uint64_t stride = nwaves * 64 * R;
    // column c's address of each MFMA tile, loaded one wavefront step ahead so
    // that the model's arithmetic overlaps the next step's HBM reads
    u64x2 ahead[R][4];
    auto load_step = [&](uint64_t b) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int tile = 0; tile < 4; ++tile) {
                const uint64_t i = b + 64 * r + 16 * tile + c;
                ahead[r][tile] = __builtin_nontemporal_load(addrs + (i < n ? i : n - 1));
            }
    };
    if (wave * 64 * R < n) load_step(wave * 64 * R);
    for (uint64_t base = wave * 64 * R; base < n; base += stride) {
        u64x2 cur[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int tile = 0; tile < 4; ++tile) cur[r][tile] = ahead[r][tile];
        if (base + stride < n) load_step(base + stride);
        uint64_t xh[R];
        uint32_t q[R], lastq[R];
        bool ok[R];
        uint64_t tk[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // the model, 16 addresses per MFMA tile; this lane's address is base + 64r + l
            float y = 0.f;
            uint64_t xhi = 0;
#pragma unroll
            for (int tile = 0; tile < 4; ++tile) {
                const float yt = mlp_infer(Rg, C, b3, cur[r][tile].x, cur[r][tile].y);
                if (g == tile) {
                    y = yt;
                    xhi = cur[r][tile].x;
                }
            }
            xh[r] = xhi;
            const uint32_t tx = (uint32_t)(xhi >> 32);
            const uint64_t p = predict_position(y, m);
            const uint32_t e0 = eps[lookup_segment(p, M)];
            // window of positions -> range of leaves (an empty segment searches
            // every leaf); positions are below m < 2^32
            uint32_t q0 = 0, q1 = last_leaf;
            if (e0 != kEmpty) {
                const uint64_t w = 2 * (uint64_t)e0 + 16;
                q0 = (uint32_t)(p > w ? p - w : 0) / LC;
                q1 = (uint32_t)min(p + w, m - 1) / LC;
            }
            // lo = q0 + the number of leaves in [q0, q1] whose top is <= tx (the
            // tops are sorted): counted over that range extended past q1 by
            // copies of tops[q1], which keeps it sorted, with the same steps in
            // every lane (no divergent loop), then clamped to the range
            uint32_t cnt = 0;
            for (uint32_t s = top; s != 0; s >>= 1) {
                const uint32_t more = cnt + s;
                cnt = tops[min(q0 + more - 1, q1)] <= tx ? more : cnt;
            }
            const uint32_t lo = q0 + min(cnt, q1 - q0 + 1);
            // verified on the tops: some leaf of the range starts at or below x's
            // top, and the leaf after the range starts above it
            ok[r] = lo > q0 && (lo <= q1 || q1 == last_leaf || tops[q1 + 1] > tx);
            const uint32_t L = lo > q0 ? lo - 1 : q0;
            q[r] = L;
            lastq[r] = tops[L];
            // the whole first key of a tied leaf; untied lanes all read key 0
            const bool tie = ok[r] && lastq[r] == tx;
            tk[r] = gkeys[tie ? t.leaf_base + L * (uint32_t)D::kLS : 0u];
        }
        // hand-off: G lanes per lookup; round u serves owner lane (u % G) * LPW + lane / G
        const int grp = l / G, j = l % G;
        uint64_t yh[T], yl[T];
        uint32_t pq[T];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const int owner = (u % G) * LPW + grp;
            yh[u] = D::shfl64(xh[u / G], owner);
            yl[u] = 0;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < R; ++r) asm volatile("" : "+v"(tk[r]));
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t tx = (uint32_t)(xh[r] >> 32);
            uint32_t L = q[r];
            if (ok[r] && lastq[r] == tx && tk[r] > xh[r]) {  // walk back over leaves whose tops tie
                --L;
                while (L > 0 && tops[L] == tx && gkeys[t.leaf_base + L * (uint32_t)D::kLS] > xh[r]) --L;
            }
            q[r] = L;
        }
#pragma unroll
        for (int u = 0; u < T; ++u) pq[u] = (uint32_t)__shfl((int)q[u / G], (u % G) * LPW + grp, 64);
        uint32_t res[T];
        D::template leaf_blocks<T>(t, gkeys, pq, yh, yl, j, l - j, 0, res);
        const int gsel = l / LPW, src = (l % LPW) * G;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t v = 0;
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const uint32_t got = (uint32_t)__shfl((int)res[r * G + k], src, 64);
                v = k == gsel ? got : v;
            }
            const uint64_t i = base + (uint64_t)r * 64 + l;
            const bool need = !ok[r] && i < n;
            const uint64_t mask = __ballot(need);
            if constexpr (QUEUE) {
                if (mask) {
                    const int first_lane = __builtin_ctzll(mask);
                    uint32_t first = 0;
                    if (l == first_lane) first = atomicAdd(fq.count, (uint32_t)__popcll(mask));
                    first = (uint32_t)__builtin_amdgcn_readlane((int)first, first_lane);
                    const uint32_t slot = first + (uint32_t)__popcll(mask & ((1ull << l) - 1ull));
                    if (need && slot < fq.cap) fq.idx[slot] = (uint32_t)i;  // cap >= n: always taken
                }
                if (ok[r] && i < n) __builtin_nontemporal_store((uint16_t)v, out + i);
            } else {
                if (need) v = t.vals[descend_lane<B, 8>(t, xh[r], 0)];
                if (i < n) __builtin_nontemporal_store((uint16_t)v, out + i);
                if (fq.count && l == 0 && mask) atomicAdd(fq.count, (uint32_t)__popcll(mask));
            }
        }
    }
}

// Leaf tops of a tree with 64-bit key slots: the high 32 bits of each leaf's first key.
template <int B>
__global__ void leaf_tops_kernel(TreeDesc t, uint32_t* __restrict__ tops, uint32_t nleaves)
{
    constexpr int LS = leaf_slots_for(B, 8);
    const auto* keys = static_cast<const uint64_t*>(t.keys);
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nleaves; q += gridDim.x * blockDim.x)
        tops[q] = (uint32_t)(keys[t.leaf_base + (uint64_t)q * LS] >> 32);
}

// Clears the fallback queue before a learned lookup (a kernel, not a memset,
// so that the sequence can be captured into a graph).
__global__ void queue_reset_kernel(uint32_t* count)
{
    if (threadIdx.x == 0) *count = 0;
}

// The tree descent for the queued lookups; adds their number to fallbacks.
template <int B, int KB>
__global__ void __launch_bounds__(kLearnBlock)
fallback_kernel(TreeDesc t, const u64x2* __restrict__ addrs, uint16_t* __restrict__ out, FallbackQueue fq,
                uint32_t* __restrict__ fallbacks)
{
    const uint32_t c = min(*fq.count, fq.cap);
    if (fallbacks && c && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(fallbacks, c);
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < c; k += gridDim.x * blockDim.x) {
        const uint32_t i = fq.idx[k];
        const u64x2 a = __builtin_nontemporal_load(addrs + i);
        __builtin_nontemporal_store(t.vals[descend_lane<B, KB>(t, a.x, a.y)], out + i);
    }
}

// Learned lookups of bursts that each name a table: tiles of 64 addresses
// (one wavefront step) never cross a burst, so every step runs one table's
// model.  A wavefront reloads the model's operands and per-row constants (80
// registers) when its tile's table changes; a table without a model is
// searched by the tree descent.
template <int B, int KB>
__global__ void __launch_bounds__(kLearnBlock)
multi_learned_kernel(const TreeDesc* __restrict__ tables, const ModelDesc* __restrict__ models, uint32_t n_tables,
                     const BurstRec* __restrict__ bursts, const uint32_t* __restrict__ count, uint32_t max_bursts,
                     uint32_t* __restrict__ fallbacks)
{
    extern __shared__ uint32_t lds_u32[];
    uint32_t* tile_off = lds_u32;                                   // max_bursts + 1
    uint32_t* part = tile_off + max_bursts + 1;                     // kLearnBlock
    auto live = [&](uint32_t tb) { return tb < n_tables && tables[tb].depth != 0; };
    const uint32_t nb = plan_burst_tiles<kLearnBlock>(bursts, count, max_bursts, 64, live, tile_off, part);
    const uint32_t total = tile_off[nb];
    const uint32_t nwaves = gridDim.x * (kLearnBlock / 64);
    const int l = threadIdx.x & 63;
    InferRegs R;
    InferConsts C;
    float b3 = 0.f;
    uint32_t loaded = 0xFFFFFFFFu;  // table whose model R and C hold
    // Each wavefront takes a contiguous run of tiles, not every nwaves-th: a
    // burst's tiles are consecutive, so the model's 80 registers of operands
    // are reloaded about once per burst instead of once per tile.
    const uint32_t wave = blockIdx.x * (kLearnBlock / 64) + (threadIdx.x >> 6);
    const uint32_t per = (total + nwaves - 1) / nwaves;
    const uint32_t first = (uint32_t)min((uint64_t)wave * per, (uint64_t)total);
    const uint32_t last = (uint32_t)min((uint64_t)first + per, (uint64_t)total);
    for (uint32_t tile = first; tile < last; ++tile) {
        const uint32_t k = burst_of_tile(tile_off, nb, tile);
        const BurstRec br = bursts[k];
        const TreeDesc& t = tables[br.table];
        const ModelDesc M = models[br.table];
        const uint64_t base = (uint64_t)(tile - tile_off[k]) * 64;
        const u64x2* addrs = br.addrs;
        uint16_t* out = static_cast<uint16_t*>(br.out);
        if (M.wb == nullptr) {  // no model: the tree descent, one lane per address
            const uint64_t i = base + l;
            if (i < br.n) {
                const u64x2 a = __builtin_nontemporal_load(addrs + i);
                __builtin_nontemporal_store(t.vals[descend_lane<B, KB>(t, a.x, a.y)], out + i);
            }
            continue;
        }
        if (br.table != loaded) {  // uniform across the wavefront
            load_infer(M.wb, R);
            load_consts(M, C);
            b3 = M.w[ob3];
            loaded = br.table;
        }
        learned_step<B, KB, false>(t, M, R, C, b3, addrs, base, br.n, out, fallbacks, FallbackQueue{});
    }
}

// Raw model output y for n addresses.
__global__ void __launch_bounds__(kLearnBlock)
predict_kernel(ModelDesc M, const u64x2* __restrict__ addrs, uint64_t n, float* __restrict__ y)
{
    InferRegs R;
    load_infer(M.wb, R);
    InferConsts C;
    load_consts(M, C);
    const float b3 = M.w[ob3];
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    const uint64_t wave = (uint64_t)blockIdx.x * (kLearnBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kLearnBlock / 64);
    // each step's address is loaded one step ahead
    u64x2 next = addrs[min(wave * 16 + c, n - 1)];
    for (uint64_t base = wave * 16; base < n; base += nwaves * 16) {
        const uint64_t i = base + c;
        const u64x2 a = next;
        next = addrs[min(base + nwaves * 16 + c, n - 1)];
        const float yt = mlp_infer(R, C, b3, a.x, a.y);
        if (g == 0 && i < n) y[i] = yt;
    }
}

// eps_acc[seg] = max over points of (|p - idx| + 1); 0 = no point.
__global__ void eps_accumulate_kernel(const float* __restrict__ y, const uint32_t* __restrict__ idx, uint64_t npts,
                                      uint64_t m, uint32_t segments, float inv_m, uint32_t* __restrict__ eps_acc)
{
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npts; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = predict_position(y[k], m);
        const uint64_t want = idx[k];
        const uint64_t err = p > want ? p - want : want - p;
        const uint32_t seg = segment_of(p, segments, m, inv_m);
        atomicMax(eps_acc + seg, (uint32_t)min(err + 1, (uint64_t)0xFFFFFFFEu));
    }
}

__global__ void eps_finalize_kernel(uint32_t* eps, uint32_t segments)
{
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < segments; s += gridDim.x * blockDim.x)
        eps[s] = eps[s] == 0 ? kEmpty : eps[s] - 1;
}

// ---------------------------------------------------------------- training
constexpr int kTrainWaves = 4;

struct TrainArgs {
    const u64x2* samples;
    const float* targets;
    const uint32_t* order;  // sample k of the batch is samples[order[first + k]] (NULL: first + k)
    uint64_t first;
    uint32_t count;         // batch size N
    float* partials;        // [gridDim.x][kParams]
};

// Gradient of mean((y - t)^2) over one batch; each workgroup writes the sum
// of its tiles' contributions to its own row of `partials` (fixed order, no
// floating-point atomics), reduced by adam_kernel.
__global__ void __launch_bounds__(64 * kTrainWaves)
grad_kernel(ModelDesc M, TrainArgs T)
{
    __shared__ float sb1[kH], sb2[kH], sw3[kH];
    __shared__ uint16_t sD2[kTrainWaves][kH][16], sD1[kTrainWaves][kH][16], sH1[kTrainWaves][kH][16];
    __shared__ uint16_t sXt[kTrainWaves][kF][16];
    __shared__ float red[kH * kH];
    stage_small(M, sb1, sb2, sw3);
    __syncthreads();
    MlpRegs R;
    load_regs(M.wb, R);
    s4 w2t[4][4];  // A operand of W2^T: W2[16kb + 4g + i][16mb + l%16]
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15, w = threadIdx.x >> 6;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) w2t[mb][kb][i] = (short)M.wb[oW2 + (16 * kb + 4 * g + i) * kH + 16 * mb + c];
    const float b3 = M.w[ob3];
    const float inv_n = 2.0f / (float)T.count;

    f4 gW2[4][4], gW1[4];
    float gb1[16], gb2[16], gw3[16], gb3 = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) gb1[k] = gb2[k] = gw3[k] = 0.f;

    const uint32_t tiles = (T.count + 15) / 16;
    for (uint32_t tile = blockIdx.x * kTrainWaves + w; tile < tiles; tile += gridDim.x * kTrainWaves) {
        const uint32_t k = tile * 16 + c;
        const bool valid = k < T.count;
        const uint64_t src = T.first + (valid ? k : 0);
        const uint64_t sidx = T.order ? T.order[src] : src;
        const u64x2 a = T.samples[sidx];
        const float target = T.targets[sidx];
        Activations A;
        const float y = mlp_forward(R, sb1, sb2, sw3, b3, a.x, a.y, A);
        const float dy = valid ? (y - target) * inv_n : 0.f;
        // feature matrix, transposed: sXt[f][column]
        const s4 xb = feature_operand(a.x, a.y);
#pragma unroll
        for (int i = 0; i < 4; ++i) sXt[w][4 * g + i][c] = (uint16_t)xb[i];
        s4 d2b[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 4 * mb + i, u = 16 * mb + 4 * g + i;
                const float h2 = A.h2[mb][i];
                const float d2 = h2 > 0.f ? sw3[u] * dy : 0.f;
                gb2[r] += d2;
                gw3[r] = fmaf(h2, dy, gw3[r]);
                const uint16_t q = f2bf(d2);
                d2b[mb][i] = (short)q;
                sD2[w][u][c] = q;
                sH1[w][u][c] = (uint16_t)A.h1b[mb][i];
            }
        }
        if (g == 0) gb3 += dy;
        // dH1^T = W2^T dZ2^T, masked by the layer-1 ReLU
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w2t[mb][kb], d2b[kb], z, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = 16 * mb + 4 * g + i;
                const float d1 = A.h1[mb][i] > 0.f ? z[i] : 0.f;
                gb1[4 * mb + i] += d1;
                sD1[w][u][c] = f2bf(d1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // dW2 += dZ2^T H1 (K = the 16 samples), dW1 += dZ1^T X
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            s4 a2, a1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a2[i] = (short)sD2[w][16 * mb + c][4 * g + i];
                a1[i] = (short)sD1[w][16 * mb + c][4 * g + i];
            }
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                s4 bh;
#pragma unroll
                for (int i = 0; i < 4; ++i) bh[i] = (short)sH1[w][16 * nb + c][4 * g + i];
                gW2[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, bh, gW2[mb][nb], 0, 0, 0);
            }
            s4 bx;
#pragma unroll
            for (int i = 0; i < 4; ++i) bx[i] = (short)sXt[w][c][4 * g + i];
            gW1[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, bx, gW1[mb], 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // per-unit vectors: sum over the 16 columns of each row group
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            gb1[r] += __shfl_xor(gb1[r], o, 64);
            gb2[r] += __shfl_xor(gb2[r], o, 64);
            gw3[r] += __shfl_xor(gw3[r], o, 64);
        }
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) gb3 += __shfl_xor(gb3, o, 64);

    // combine the waves in a fixed order, one parameter block at a time
    float* dst = T.partials + (size_t)blockIdx.x * kParams;
    // W2 (64 x 64)
    for (int ww = 0; ww < kTrainWaves; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int idx = (16 * mb + 4 * g + i) * kH + 16 * nb + c;
                        red[idx] = (ww == 0 ? 0.f : red[idx]) + gW2[mb][nb][i];
                    }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) dst[oW2 + i] = red[i];
    __syncthreads();
    // W1 (64 x 16), b1, b2, w3, b3 packed into red[]
    for (int ww = 0; ww < kTrainWaves; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int idx = (16 * mb + 4 * g + i) * kF + c;
                    red[idx] = (ww == 0 ? 0.f : red[idx]) + gW1[mb][i];
                }
            if (c == 0) {
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int u = 16 * mb + 4 * g + i, r = 4 * mb + i;
                        red[1024 + u] = (ww == 0 ? 0.f : red[1024 + u]) + gb1[r];
                        red[1088 + u] = (ww == 0 ? 0.f : red[1088 + u]) + gb2[r];
                        red[1152 + u] = (ww == 0 ? 0.f : red[1152 + u]) + gw3[r];
                    }
            }
            if (l == 0) red[1216] = (ww == 0 ? 0.f : red[1216]) + gb3;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < kH * kF; i += blockDim.x) dst[oW1 + i] = red[i];
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        dst[ob1 + i] = red[1024 + i];
        dst[ob2 + i] = red[1088 + i];
        dst[ow3 + i] = red[1152 + i];
    }
    if (threadIdx.x == 0) dst[ob3] = red[1216];
}

// Sum the workgroup partials in order; optionally apply one Adam step to the
// float32 master weights and refresh the bfloat16 copy.
__global__ void adam_kernel(const float* __restrict__ partials, uint32_t nparts, float* __restrict__ grad_out,
                            float* __restrict__ w, float* __restrict__ m1, float* __restrict__ m2,
                            uint16_t* __restrict__ wb, int apply, float lr, float beta1, float beta2, float eps,
                            float corr1, float corr2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    float gsum = 0.f;
    for (uint32_t k = 0; k < nparts; ++k) gsum += partials[(size_t)k * kParams + p];
    if (grad_out) grad_out[p] = gsum;
    if (!apply) return;
    const float a = beta1 * m1[p] + (1.f - beta1) * gsum;
    const float b = beta2 * m2[p] + (1.f - beta2) * gsum * gsum;
    m1[p] = a;
    m2[p] = b;
    const float upd = (a / corr1) / (sqrtf(b / corr2) + eps);
    const float nw = w[p] - lr * upd;
    w[p] = nw;
    wb[p] = f2bf(nw);
}

// ------------------------------------------------------------- host side
struct LearnedModel {
    float* w = nullptr;      // master weights
    float* m1 = nullptr;     // Adam first moment
    float* m2 = nullptr;     // Adam second moment
    uint16_t* wb = nullptr;  // bf16 copy
    uint32_t* eps = nullptr;
    uint32_t segments = 0;
    float seg_scale = 0.f;  // segments / m
    float* partials = nullptr;
    uint32_t max_parts = 256;
    uint64_t adam_steps = 0;
    bool has_eps = false;
    uint32_t* leaf_tops = nullptr;  // 64-bit key slots: top 32 bits of each leaf's first key
    uint32_t nleaves = 0;
};

namespace {

// The two kernels of a learned lookup for one (fanout, key width).
struct LearnedFns {
    void* lookup = nullptr;
    void* fallback = nullptr;
    void* direct = nullptr;  // the lookup with fallbacks descended in place (no queue)
};

template <int B, int KB>
LearnedFns learned_fns()
{
    return {reinterpret_cast<void*>(learned_kernel<B, KB, true>), reinterpret_cast<void*>(fallback_kernel<B, KB>),
            reinterpret_cast<void*>(learned_kernel<B, KB, false>)};
}

template <int B>
LearnedFns learned_by_kb(int kb)
{
    return kb == 4 ? learned_fns<B, 4>() : kb == 8 ? learned_fns<B, 8>() : learned_fns<B, 16>();
}

// The leaf-tops learned kernel: B in {8, 16} (128-byte leaves, 4 lanes of one
// 32-byte block each), one lookup per lane and 768 threads.  The leaf tops
// take most of the LDS, so one workgroup runs per CU; at 168 VGPRs a
// 768-thread workgroup gives 3 waves per SIMD.  Two lookups per lane need 228
// VGPRs, so only 512 threads (2 waves per SIMD): 30.9 against 33.1 GLPS on
// the 200k backbone FIB (2^26 addresses), 26.8 against 28.2 on the tiny one.
// 1024 threads would leave 128 VGPRs, and the model's registers spill.
constexpr int kLearnTopsBlock = 768;

// planb_lookup_learned calls of fewer lookups run the direct (queue-free)
// kernel: one launch, no allocation.  Measured crossovers (200k backbone and
// 1k tiny FIBs): the leaf-tops kernel's in-place fallbacks are rare and short
// (2^20 lookups: 58.6 against 66.0 us queued; 2^22: 146 against 138), the
// other kernel's whole-tree descents of 16-byte keys cost more (2^16: 20.5
// against 31.9 us; 2^20: 103 against 93).
constexpr uint64_t kLearnedDirectMaxTops = 1ull << 21;
constexpr uint64_t kLearnedDirectMax = 1ull << 18;

template <bool QUEUE>
void* pick_learned_tops(int B)
{
    return B == 8    ? reinterpret_cast<void*>(learned_tops_kernel<8, 2, 1, kLearnTopsBlock, QUEUE>)
           : B == 16 ? reinterpret_cast<void*>(learned_tops_kernel<16, 4, 1, kLearnTopsBlock, QUEUE>)
                     : nullptr;
}

LearnedFns pick_learned(int B, int kb)
{
    switch (B) {
    case 8: return learned_by_kb<8>(kb);
    case 16: return learned_by_kb<16>(kb);
    case 32: return learned_by_kb<32>(kb);
    default: return {};
    }
}

ModelDesc model_desc(const LearnedModel* L)
{
    return ModelDesc{L->wb, L->w, L->eps, L->segments, L->seg_scale};
}

int ensure_model(planb_fib_t* f, uint32_t segments)
{
    if (segments == 0) segments = 4096;
    // the learned kernels keep positions in 32 bits
    if (f->desc.m_minus_1 >= 0xFFFFFFFFull) return fail(PLANB_ERANGE, "a learned model needs fewer than 2^32 intervals");
    LearnedModel* L = f->learned;
    if (L && L->segments != segments) {
        release_learned(f);
        L = nullptr;
    }
    if (L) return PLANB_OK;
    L = new (std::nothrow) LearnedModel();
    if (!L) return fail(PLANB_ENOMEM, "out of host memory");
    f->learned = L;
    L->segments = segments;
    L->seg_scale = (float)((double)segments / (double)(f->desc.m_minus_1 + 1));
    hipError_t e;
    auto get = [&](auto** p, size_t bytes) { return fib_alloc(f->device, reinterpret_cast<void**>(p), bytes); };
    if ((e = get(&L->w, kParams * 4)) != hipSuccess || (e = get(&L->m1, kParams * 4)) != hipSuccess ||
        (e = get(&L->m2, kParams * 4)) != hipSuccess || (e = get(&L->wb, kParams * 2)) != hipSuccess ||
        (e = get(&L->eps, (size_t)segments * 4)) != hipSuccess ||
        (e = get(&L->partials, (size_t)L->max_parts * kParams * 4)) != hipSuccess) {
        release_learned(f);
        return fail(PLANB_ENOMEM, std::string("device allocation: ") + hipGetErrorString(e));
    }
    if (f->desc.key_bytes == 8 && f->desc.depth >= 1) {  // the tree never changes: its leaf tops are built once
        const TreeDesc& t = f->desc;
        L->nleaves = t.last[t.depth - 1] + 1;
        if ((e = get(&L->leaf_tops, (size_t)L->nleaves * 4)) != hipSuccess) {
            release_learned(f);
            return fail(PLANB_ENOMEM, std::string("device allocation: ") + hipGetErrorString(e));
        }
        const unsigned grid = std::min<unsigned>((L->nleaves + 255) / 256, 1024);
        switch (t.fanout) {
        case 8: hipLaunchKernelGGL(leaf_tops_kernel<8>, dim3(grid), dim3(256), 0, nullptr, t, L->leaf_tops, L->nleaves); break;
        case 16: hipLaunchKernelGGL(leaf_tops_kernel<16>, dim3(grid), dim3(256), 0, nullptr, t, L->leaf_tops, L->nleaves); break;
        case 32: hipLaunchKernelGGL(leaf_tops_kernel<32>, dim3(grid), dim3(256), 0, nullptr, t, L->leaf_tops, L->nleaves); break;
        default: break;
        }
        if ((e = hipGetLastError()) == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) {
            release_learned(f);
            return fail_hip(e, "building the leaf tops");
        }
    }
    return PLANB_OK;
}

int upload_params(LearnedModel* L, const float* host)
{
    std::vector<uint16_t> b(kParams);
    for (int i = 0; i < kParams; ++i) b[i] = f2bf(host[i]);
    hipError_t e;
    if ((e = hipMemcpy(L->w, host, kParams * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(L->wb, b.data(), kParams * 2, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(L->m1, 0, kParams * 4)) != hipSuccess || (e = hipMemset(L->m2, 0, kParams * 4)) != hipSuccess ||
        (e = hipMemset(L->eps, 0xFF, (size_t)L->segments * 4)) != hipSuccess)
        return fail_hip(e, "uploading model parameters");
    L->adam_steps = 0;
    L->has_eps = false;
    return PLANB_OK;
}

// Seeded initialisation: W ~ U(-1/sqrt(fan_in), +1/sqrt(fan_in)), biases 0,
// b3 = 0.5 (the middle of the position range).
std::vector<float> init_params(uint64_t seed)
{
    std::mt19937_64 rng(seed);
    std::vector<float> p(kParams, 0.f);
    auto fill = [&](int off, int count, float bound) {
        std::uniform_real_distribution<float> d(-bound, bound);
        for (int i = 0; i < count; ++i) p[off + i] = d(rng);
    };
    fill(oW1, kH * kF, 1.0f / std::sqrt((float)kF));
    fill(oW2, kH * kH, 1.0f / std::sqrt((float)kH));
    fill(ow3, kH, 1.0f / std::sqrt((float)kH));
    p[ob3] = 0.5f;
    return p;
}

// Training / error-table points: for every interval its first and last
// address and kInterior addresses drawn uniformly inside it (seeded), each
// labelled with the interval index.  The interior draws give the low address
// bytes the same spread that lookup traffic has, so the model learns that
// they do not move the position.
constexpr int kPointsPerInterval = 4;

void boundary_points(const Intervals& iv, uint64_t seed, std::vector<U128>* pts, std::vector<uint32_t>* idx)
{
    using u128 = unsigned __int128;
    const size_t m = iv.starts.size();
    pts->resize(kPointsPerInterval * m);
    idx->resize(kPointsPerInterval * m);
    std::mt19937_64 rng(seed * 0x2545F4914F6CDD1Dull + 0x6A09E667F3BCC909ull);
    auto to_u = [](U128 v) { return ((u128)v.hi << 64) | v.lo; };
    auto from_u = [](u128 v) { return U128{(uint64_t)(v >> 64), (uint64_t)v}; };
    for (size_t i = 0; i < m; ++i) {
        const u128 s = to_u(iv.starts[i]);
        const u128 last = i + 1 < m ? to_u(iv.starts[i + 1]) - 1 : ~(u128)0;
        const u128 span = last - s;  // size - 1
        U128* out = pts->data() + kPointsPerInterval * i;
        out[0] = from_u(s);
        out[1] = from_u(last);
        for (int k = 2; k < kPointsPerInterval; ++k) {
            const u128 r = ((u128)rng() << 64) | rng();
            out[k] = from_u(span == ~(u128)0 ? r : s + r % (span + 1));
        }
        for (int k = 0; k < kPointsPerInterval; ++k) (*idx)[kPointsPerInterval * i + k] = (uint32_t)i;
    }
}

// Segments actually used for m intervals: at most the requested count and at
// least 64 positions per segment (narrower segments see too few points).
uint32_t effective_segments(uint32_t requested, uint64_t m)
{
    const uint64_t cap = std::max<uint64_t>(1, m / 64);
    return (uint32_t)std::min<uint64_t>(requested ? requested : 4096, cap);
}

int launch_grad(const LearnedModel* L, const TrainArgs& base, uint32_t* parts_used, hipStream_t st)
{
    const uint32_t tiles = (base.count + 15) / 16;
    uint32_t grid = (tiles + kTrainWaves - 1) / kTrainWaves;
    grid = std::max(1u, std::min(grid, L->max_parts));
    TrainArgs T = base;
    T.partials = L->partials;
    hipLaunchKernelGGL(grad_kernel, dim3(grid), dim3(64 * kTrainWaves), 0, st, model_desc(L), T);
    *parts_used = grid;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "gradient launch");
}

int launch_adam(LearnedModel* L, uint32_t parts, float* grad_out, bool apply, float lr, hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.f, c2 = 1.f;
    if (apply) {
        ++L->adam_steps;
        c1 = 1.f - (float)std::pow(0.9, (double)L->adam_steps);
        c2 = 1.f - (float)std::pow(0.999, (double)L->adam_steps);
    }
    hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, st, L->partials, parts, grad_out, L->w,
                       L->m1, L->m2, L->wb, apply ? 1 : 0, lr, b1, b2, 1e-8f, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "adam launch");
}

int build_eps(planb_fib_t* f, const u64x2* d_pts, const uint32_t* d_idx, uint64_t npts, float* d_y, hipStream_t st)
{
    LearnedModel* L = f->learned;
    const uint64_t m = f->iv.starts.size();
    hipLaunchKernelGGL(predict_kernel, dim3((unsigned)std::min<uint64_t>((npts + 63) / 64, 4096)), dim3(kLearnBlock), 0,
                       st, model_desc(L), d_pts, npts, d_y);
    hipError_t e = hipMemsetAsync(L->eps, 0, (size_t)L->segments * 4, st);
    if (e != hipSuccess) return fail_hip(e, "clearing the epsilon table");
    hipLaunchKernelGGL(eps_accumulate_kernel, dim3((unsigned)std::min<uint64_t>((npts + 255) / 256, 4096)), dim3(256), 0,
                       st, d_y, d_idx, npts, m, L->segments, 1.0f / (float)m, L->eps);
    hipLaunchKernelGGL(eps_finalize_kernel, dim3((L->segments + 255) / 256), dim3(256), 0, st, L->eps, L->segments);
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "epsilon table launch");
    L->has_eps = true;
    return PLANB_OK;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes); }
};

}  // namespace

void release_learned(planb_fib_t* f)
{
    LearnedModel* L = f->learned;
    if (!L) return;
    // lookups already enqueued may still read the model: freed after them
    free_after(f->uses, f->device,
               {(void*)L->w, (void*)L->m1, (void*)L->m2, (void*)L->wb, (void*)L->eps, (void*)L->partials,
                (void*)L->leaf_tops});
    delete L;
    f->learned = nullptr;
}

size_t learned_model_bytes(uint32_t segments, uint64_t nleaves)
{
    if (segments == 0) segments = 4096;
    return (size_t)kParams * (3 * 4 + 2) + (size_t)segments * 4 + (size_t)LearnedModel{}.max_parts * kParams * 4 +
           (size_t)nleaves * 4;
}

ModelDesc ready_model_desc(const planb_fib_t* f)
{
    if (!f || !f->learned || !f->learned->has_eps) return ModelDesc{nullptr, nullptr, nullptr, 0, 0.f};
    return model_desc(f->learned);
}

namespace {

template <int B, int KB>
struct MultiLearnedKernel {
    static const void* get() { return reinterpret_cast<const void*>(multi_learned_kernel<B, KB>); }
};

template <int B>
const void* multi_learned_by_kb(int kb)
{
    return kb == 4 ? MultiLearnedKernel<B, 4>::get() : kb == 8 ? MultiLearnedKernel<B, 8>::get()
                                                               : MultiLearnedKernel<B, 16>::get();
}

}  // namespace

int plan_multi_learned(int fanout, int kb, uint32_t max_bursts, MultiLaunch* L)
{
    const void* fn = nullptr;
    switch (fanout) {
    case 8: fn = multi_learned_by_kb<8>(kb); break;
    case 16: fn = multi_learned_by_kb<16>(kb); break;
    case 32: fn = multi_learned_by_kb<32>(kb); break;
    default: return fail(PLANB_EINVAL, "no learned multi-FIB kernel for this fanout");
    }
    DevProps p;
    hipError_t e = dev_props(&p);
    if (e != hipSuccess) return fail_hip(e, "device properties");
    L->fn = fn;
    L->block = kLearnBlock;
    L->lds = ((size_t)max_bursts + 1 + kLearnBlock) * 4;
    if (L->lds > (size_t)p.max_lds) return fail(PLANB_ERANGE, "too many bursts per launch for the LDS");
    int nb = 1;
    if ((e = occupancy(fn, kLearnBlock, L->lds, &nb)) != hipSuccess) return fail_hip(e, "occupancy");
    L->grid = (unsigned)(p.cus * nb);
    return PLANB_OK;
}

hipError_t launch_multi_learned(const MultiLaunch& L, const TreeDesc* tables, const ModelDesc* models,
                                uint32_t n_tables, const BurstRec* bursts, const uint32_t* count,
                                uint32_t max_bursts, uint32_t* fallbacks, hipStream_t stream)
{
    void* args[] = {&tables, &models, &n_tables, &bursts, &count, &max_bursts, &fallbacks};
    return hipLaunchKernel(L.fn, dim3(L.grid), dim3(L.block), args, L.lds, stream);
}

// ---------------------------------------------------------------- learned lookup launch
constexpr size_t kQueueHeaderBytes = 256;  // the counter, then the entries (256-byte aligned)

// The fallback queue of planb_lookup_learned_noalloc: a fixed device array
// (per GPU, for the life of the process) instead of an allocation.  Host code
// never passes `scratch` itself to a kernel: each device's address of it comes
// from hipGetSymbolAddress (static_queue).
constexpr size_t kStaticQueueEntries = size_t(1) << 22;  // 16 MiB of entries
static __device__ __align__(256) uint32_t scratch[kQueueHeaderBytes / 4 + kStaticQueueEntries];

namespace {

std::mutex g_static_mu;
std::vector<uint32_t*> g_static_ptr;  // by device ordinal; null until looked up

// Address of `scratch` on `device` (the current device), looked up once per device.
int static_queue(int device, uint32_t** out)
{
    std::lock_guard<std::mutex> lk(g_static_mu);
    if ((int)g_static_ptr.size() <= device) g_static_ptr.resize(device + 1, nullptr);
    if (!g_static_ptr[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(PLANB_EDEVICE, std::string("looking up the static fallback queue: ") + hipGetErrorString(e));
        }
        g_static_ptr[device] = static_cast<uint32_t*>(ptr);
    }
    *out = g_static_ptr[device];
    return PLANB_OK;
}

int learned_check(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, const uint16_t* out,
                  const uint32_t* fallback_count)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    if (!fib->learned || !fib->learned->has_eps) return fail(PLANB_EINVAL, "the FIB has no trained model");
    if (n == 0) return PLANB_OK;
    if (n >= (1ull << 32)) return fail(PLANB_ERANGE, "batch too large (n must be < 2^32)");
    if (!addrs || !out) return fail(PLANB_EINVAL, "NULL device pointer");
    if (reinterpret_cast<uintptr_t>(addrs) % 16 || reinterpret_cast<uintptr_t>(out) % 2 ||
        reinterpret_cast<uintptr_t>(fallback_count) % 4)
        return fail(PLANB_EINVAL, "misaligned pointer");
    return check_current_device(fib);
}

// Whether a learned lookup on this FIB runs the leaf-tops kernel: 64-bit key
// slots, and the leaf tops and error table fit a workgroup's LDS.
bool learned_uses_tops(const planb_fib_t* fib)
{
    const LearnedModel* LM = fib->learned;
    DevProps p;
    if (!LM->leaf_tops || dev_props(&p) != hipSuccess || !pick_learned_tops<true>((int)fib->desc.fanout)) return false;
    return learned_tops_lds_bytes(LM->nleaves, LM->segments) <= (size_t)p.max_lds;
}

// Reset the queue, run the learned lookup, then the tree descent for the
// queued lookups; fq.cap >= n.  With fq.count null (direct), one launch:
// failing lookups descend the tree in place, counted in fallback_count.
int launch_learned(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint16_t* out,
                   uint32_t* fallback_count, FallbackQueue fq, hipStream_t st)
{
    const bool direct = fq.count == nullptr;
    if (direct) fq = FallbackQueue{fallback_count, nullptr, 0};
    const LearnedFns fns = pick_learned((int)fib->desc.fanout, (int)fib->desc.key_bytes);
    if (!fns.lookup) return fail(PLANB_EINVAL, "no learned kernel for this fanout");
    DevProps p;
    hipError_t e = dev_props(&p);
    if (e != hipSuccess) return fail_hip(e, "device properties");
    TreeDesc t = fib->desc;
    const LearnedModel* LM = fib->learned;
    ModelDesc M = model_desc(LM);
    const u64x2* a = reinterpret_cast<const u64x2*>(addrs);
    uint64_t nn = n;
    // the leaf-tops kernel when the tree has 64-bit key slots and its leaf tops
    // and error table fit a workgroup's LDS, else the window search over the
    // leaf keys
    const int R = 1, bs = kLearnTopsBlock;
    void* tops_fn = !learned_uses_tops(fib) ? nullptr
                    : direct                 ? pick_learned_tops<false>((int)t.fanout)
                                             : pick_learned_tops<true>((int)t.fanout);
    void* lookup_fn = direct ? fns.direct : fns.lookup;
    const size_t tops_lds = learned_tops_lds_bytes(LM->nleaves, LM->segments);
    if (!direct) hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, fq.count);
    if (tops_fn) {
        int nb = 1;
        if ((e = occupancy(tops_fn, bs, tops_lds, &nb)) != hipSuccess) return fail_hip(e, "occupancy");
        const uint64_t per_block = (uint64_t)(bs / 64) * 64 * R;
        const unsigned grid = (unsigned)std::min<uint64_t>((n + per_block - 1) / per_block, (uint64_t)p.cus * nb);
        LeafTops lt{LM->leaf_tops, LM->nleaves};
        void* args[] = {&t, &M, &lt, &a, &nn, &out, &fq};
        if ((e = hipLaunchKernel(tops_fn, dim3(grid), dim3(bs), args, tops_lds, st)) != hipSuccess)
            return fail_hip(e, "learned lookup launch");
    } else {
        int nb = 1;
        if ((e = occupancy(lookup_fn, kLearnBlock, 0, &nb)) != hipSuccess) return fail_hip(e, "occupancy");
        const uint64_t want = (n + (kLearnBlock / 64) * 64 - 1) / ((kLearnBlock / 64) * 64);
        const unsigned grid = (unsigned)std::min<uint64_t>(want, (uint64_t)p.cus * nb);
        void* args[] = {&t, &M, &a, &nn, &out, &fq};
        if ((e = hipLaunchKernel(lookup_fn, dim3(grid), dim3(kLearnBlock), args, 0, st)) != hipSuccess)
            return fail_hip(e, "learned lookup launch");
    }
    if (!direct) {
        // the queue's length is known only on the device: a fixed grid walks it
        const unsigned fgrid = (unsigned)std::min<uint64_t>((n + kLearnBlock - 1) / kLearnBlock, (uint64_t)p.cus * 2);
        void* fargs[] = {&t, &a, &out, &fq, &fallback_count};
        if ((e = hipLaunchKernel(fns.fallback, dim3(fgrid), dim3(kLearnBlock), fargs, 0, st)) != hipSuccess)
            return fail_hip(e, "fallback launch");
    }
    if ((e = hipGetLastError()) != hipSuccess) return fail_hip(e, "learned lookup launch");
    note_use(fib->uses, st);
    return PLANB_OK;
}

}  // namespace

}  // namespace planb

using namespace planb;

extern "C" {

int planb_model_set_params(planb_fib_t* fib, const float* params, uint32_t segments)
{
    if (!fib || !params) return fail(PLANB_EINVAL, "NULL argument");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK || (rc = ensure_model(fib, segments ? segments : 4096)) != PLANB_OK) return rc;
    return upload_params(fib->learned, params);
}

int planb_model_get_params(const planb_fib_t* fib, float* params)
{
    if (!fib || !params) return fail(PLANB_EINVAL, "NULL argument");
    if (!fib->learned) return fail(PLANB_EINVAL, "the FIB has no model");
    hipError_t e = hipMemcpy(params, fib->learned->w, kParams * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "reading parameters");
}

int planb_model_num_params(void) { return kParams; }

int planb_model_predict(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, float* y, void* stream)
{
    if (!fib || (n && (!addrs || !y))) return fail(PLANB_EINVAL, "NULL argument");
    if (!fib->learned) return fail(PLANB_EINVAL, "the FIB has no model");
    if (n == 0) return PLANB_OK;
    if (reinterpret_cast<uintptr_t>(addrs) % 16 || reinterpret_cast<uintptr_t>(y) % 4)
        return fail(PLANB_EINVAL, "misaligned pointer");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    hipLaunchKernelGGL(predict_kernel, dim3((unsigned)std::min<uint64_t>((n + 63) / 64, 8192)), dim3(kLearnBlock), 0,
                       static_cast<hipStream_t>(stream), model_desc(fib->learned),
                       reinterpret_cast<const u64x2*>(addrs), (uint64_t)n, y);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) note_use(fib->uses, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "predict launch");
}

int planb_model_grad(planb_fib_t* fib, const planb_addr_t* samples, const float* targets, size_t n, float* grad,
                     void* stream)
{
    if (!fib || !samples || !targets || !grad || n == 0) return fail(PLANB_EINVAL, "bad argument");
    if (!fib->learned) return fail(PLANB_EINVAL, "the FIB has no model");
    if (n >= (1ull << 31)) return fail(PLANB_ERANGE, "too many samples");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    TrainArgs T{reinterpret_cast<const u64x2*>(samples), targets, nullptr, 0, (uint32_t)n, nullptr};
    uint32_t parts = 0;
    if ((rc = launch_grad(fib->learned, T, &parts, static_cast<hipStream_t>(stream))) != PLANB_OK) return rc;
    rc = launch_adam(fib->learned, parts, grad, false, 0.f, static_cast<hipStream_t>(stream));
    if (rc == PLANB_OK) note_use(fib->uses, static_cast<hipStream_t>(stream));
    return rc;
}

int planb_model_adam(planb_fib_t* fib, const float* grad, float lr, void* stream)
{
    if (!fib || !grad) return fail(PLANB_EINVAL, "NULL argument");
    if (!fib->learned) return fail(PLANB_EINVAL, "the FIB has no model");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(fib->learned->partials, grad, kParams * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "copying the gradient");
    const int rc2 = launch_adam(fib->learned, 1, nullptr, true, lr, st);
    if (rc2 == PLANB_OK) note_use(fib->uses, st);
    return rc2;
}

int planb_model_build_eps(planb_fib_t* fib, void* stream)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    if (!fib->learned) return fail(PLANB_EINVAL, "the FIB has no model");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    std::vector<U128> pts;
    std::vector<uint32_t> idx;
    boundary_points(fib->iv, 1, &pts, &idx);
    DevBuf dp, di, dy;
    hipError_t e;
    if ((e = dp.alloc(pts.size() * 16)) != hipSuccess || (e = di.alloc(idx.size() * 4)) != hipSuccess ||
        (e = dy.alloc(idx.size() * 4)) != hipSuccess)
        return fail(PLANB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((e = hipMemcpyAsync(dp.p, pts.data(), pts.size() * 16, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(di.p, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
        return fail_hip(e, "uploading boundary points");
    rc = build_eps(fib, static_cast<const u64x2*>(dp.p), static_cast<const uint32_t*>(di.p), pts.size(),
                   static_cast<float*>(dy.p), st);
    if (rc != PLANB_OK) return rc;
    e = hipStreamSynchronize(st);
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "epsilon table");
}

int planb_model_get_eps(const planb_fib_t* fib, uint32_t* eps, uint32_t cap)
{
    if (!fib || !eps) return fail(PLANB_EINVAL, "NULL argument");
    if (!fib->learned) return fail(PLANB_EINVAL, "the FIB has no model");
    const uint32_t n = std::min(cap, fib->learned->segments);
    hipError_t e = hipMemcpy(eps, fib->learned->eps, (size_t)n * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? (int)n : fail_hip(e, "reading the epsilon table");
}

int planb_model_set_eps(planb_fib_t* fib, const uint32_t* eps, uint32_t n)
{
    if (!fib || !eps) return fail(PLANB_EINVAL, "NULL argument");
    if (!fib->learned) return fail(PLANB_EINVAL, "the FIB has no model");
    if (n != fib->learned->segments) return fail(PLANB_EINVAL, "segment count differs from the model's");
    hipError_t e = hipMemcpy(fib->learned->eps, eps, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "writing the epsilon table");
    fib->learned->has_eps = true;
    return PLANB_OK;
}

int planb_train(planb_fib_t* fib, const planb_train_cfg_t* cfg_in, void* stream, planb_train_report_t* report)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    planb_train_cfg_t cfg{};
    if (cfg_in) cfg = *cfg_in;
    const uint64_t npts_all = kPointsPerInterval * (uint64_t)fib->iv.starts.size();
    if (cfg.batch == 0)  // about 32 steps per epoch, 64..4096 points per step
        cfg.batch = (uint32_t)std::min<uint64_t>(4096, std::max<uint64_t>(64, npts_all / 32 / 16 * 16));
    if (cfg.epochs == 0) {  // about 30,000 Adam steps in all (about 1.4 s for 400k intervals)
        const uint64_t per_epoch = (npts_all + cfg.batch - 1) / cfg.batch;
        cfg.epochs = (uint32_t)std::min<uint64_t>(400, std::max<uint64_t>(8, (30000 + per_epoch - 1) / per_epoch));
    }
    if (cfg.lr <= 0.f) cfg.lr = 3e-3f;
    cfg.segments = effective_segments(cfg.segments, fib->iv.starts.size());
    if (cfg.batch % 16) return fail(PLANB_EINVAL, "batch must be a multiple of 16");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK || (rc = ensure_model(fib, cfg.segments)) != PLANB_OK) return rc;
    LearnedModel* L = fib->learned;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<float> p0 = init_params(cfg.seed);
    if ((rc = upload_params(L, p0.data())) != PLANB_OK) return rc;
    std::vector<U128> pts;
    std::vector<uint32_t> idx;
    boundary_points(fib->iv, cfg.seed, &pts, &idx);
    const uint64_t npts = pts.size(), m = fib->iv.starts.size();
    std::vector<float> tgt(npts);
    for (uint64_t k = 0; k < npts; ++k) tgt[k] = (float)(((double)idx[k] + 0.5) / (double)m);
    DevBuf dp, di, dt, dord, dy;
    hipError_t e;
    if ((e = dp.alloc(npts * 16)) != hipSuccess || (e = di.alloc(npts * 4)) != hipSuccess ||
        (e = dt.alloc(npts * 4)) != hipSuccess || (e = dord.alloc(npts * 4)) != hipSuccess ||
        (e = dy.alloc(npts * 4)) != hipSuccess)
        return fail(PLANB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((e = hipMemcpyAsync(dp.p, pts.data(), npts * 16, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(di.p, idx.data(), npts * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(dt.p, tgt.data(), npts * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
        return fail_hip(e, "uploading training points");
    std::vector<uint32_t> order(npts);
    for (uint64_t k = 0; k < npts; ++k) order[k] = (uint32_t)k;
    std::mt19937_64 rng(cfg.seed ^ 0x9E3779B97F4A7C15ull);
    uint32_t steps = 0;
    for (uint32_t ep = 0; ep < cfg.epochs; ++ep) {
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail_hip(e, "training");
        std::shuffle(order.begin(), order.end(), rng);
        if ((e = hipMemcpyAsync(dord.p, order.data(), npts * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail_hip(e, "uploading the sample order");
        // cosine decay of the step size over the whole run
        for (uint64_t first = 0; first < npts; first += cfg.batch) {
            const uint32_t cnt = (uint32_t)std::min<uint64_t>(cfg.batch, npts - first);
            const double prog = (double)steps / std::max(1.0, (double)cfg.epochs * ((npts + cfg.batch - 1) / cfg.batch));
            const float lr = (float)(cfg.lr * (0.02 + 0.98 * 0.5 * (1.0 + std::cos(3.141592653589793 * prog))));
            TrainArgs T{static_cast<const u64x2*>(dp.p), static_cast<const float*>(dt.p),
                        static_cast<const uint32_t*>(dord.p), first, cnt, nullptr};
            uint32_t parts = 0;
            if ((rc = launch_grad(L, T, &parts, st)) != PLANB_OK) return rc;
            if ((rc = launch_adam(L, parts, nullptr, true, lr, st)) != PLANB_OK) return rc;
            ++steps;
        }
    }
    if ((rc = build_eps(fib, static_cast<const u64x2*>(dp.p), static_cast<const uint32_t*>(di.p), npts,
                        static_cast<float*>(dy.p), st)) != PLANB_OK)
        return rc;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail_hip(e, "training");
    if (report) {
        std::memset(report, 0, sizeof(*report));
        std::vector<float> y(npts);
        std::vector<uint32_t> eps(L->segments);
        if ((e = hipMemcpy(y.data(), dy.p, npts * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(eps.data(), L->eps, (size_t)L->segments * 4, hipMemcpyDeviceToHost)) != hipSuccess)
            return fail_hip(e, "reading the training report");
        double se = 0.0;
        for (uint64_t k = 0; k < npts; ++k) se += (double)(y[k] - tgt[k]) * (double)(y[k] - tgt[k]);
        report->final_loss = (float)(se / (double)npts);
        report->steps = steps;
        double sum = 0.0;
        uint32_t used = 0;
        for (uint32_t s = 0; s < L->segments; ++s) {
            if (eps[s] == kEmpty) {
                ++report->empty_segments;
                continue;
            }
            report->max_eps = std::max(report->max_eps, eps[s]);
            sum += eps[s];
            ++used;
        }
        report->mean_eps = used ? (float)(sum / used) : 0.f;
        report->seconds =
            (float)std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return PLANB_OK;
}

int planb_lookup_learned(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint16_t* out,
                         uint32_t* fallback_count, void* stream)
{
    int rc = learned_check(fib, addrs, n, out, fallback_count);
    if (rc != PLANB_OK || n == 0) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // Small calls run one kernel that descends the tree in place for its few
    // failing lookups: the queue's allocation and two more launches would
    // cost them more than a wavefront waiting for one lane's descent.
    if (n < (learned_uses_tops(fib) ? kLearnedDirectMaxTops : kLearnedDirectMax))
        return launch_learned(fib, addrs, n, out, fallback_count, FallbackQueue{}, st);
    // the fallback queue: a counter and one entry per lookup, from the
    // stream-ordered pool (allocated and freed in stream order: no host wait)
    void* scratch = nullptr;
    const size_t bytes = kQueueHeaderBytes + (size_t)n * 4;
    hipError_t e = hipMallocAsync(&scratch, bytes, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PLANB_ENOMEM, std::string("fallback queue (hipMallocAsync): ") + hipGetErrorString(e));
    }
    FallbackQueue fq{static_cast<uint32_t*>(scratch),
                     reinterpret_cast<uint32_t*>(static_cast<char*>(scratch) + kQueueHeaderBytes), (uint32_t)n};
    rc = launch_learned(fib, addrs, n, out, fallback_count, fq, st);
    e = hipFreeAsync(scratch, st);
    if (rc == PLANB_OK && e != hipSuccess) rc = fail_hip(e, "freeing the fallback queue");
    return rc;
}

int planb_lookup_learned_noalloc(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint16_t* out,
                                 uint32_t* fallback_count, void* stream)
{
    int rc = learned_check(fib, addrs, n, out, fallback_count);
    if (rc != PLANB_OK || n == 0) return rc;
    if (n > kStaticQueueEntries)
        return fail(PLANB_ERANGE, "planb_lookup_learned_noalloc takes at most " + std::to_string(kStaticQueueEntries) +
                                      " lookups per call (its fallback queue is a fixed device array); got " +
                                      std::to_string(n));
    uint32_t* base = nullptr;
    if ((rc = static_queue(fib->device, &base)) != PLANB_OK) return rc;
    FallbackQueue fq{base, base + kQueueHeaderBytes / 4, (uint32_t)n};
    return launch_learned(fib, addrs, n, out, fallback_count, fq, static_cast<hipStream_t>(stream));
}

}  // extern "C"
