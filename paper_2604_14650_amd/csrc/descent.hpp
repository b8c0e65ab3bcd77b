// One wavefront step of the batched tree descent, shared by the plain,
// multi-batch (persistent) and multi-FIB kernels.
//
// This is the search of the PlanB paper's Section 3 (Algorithm 1 and Listing 1)
// mapped onto a wave64: G = B / KPL lanes cooperate on one lookup.  Each lane
// compares KPL keys of the current node with the address x (arranged so that a
// group's loads are contiguous), the group adds its counts with DPP, and the
// count c of keys <= x selects child q*B + c.  At leaf q (kLC keys and their
// next hops) the interval index is q*kLC + c - 1.  Node indices are clamped to each level's last allocated
// node, which only alters the path of an address equal to the sentinel padding
// (all ones in the compared width); that address's answer is the last interval.
#pragma once

#include <type_traits>

#include "device.hpp"

namespace planb {

template <int B, int KPL, int R, int KB, bool BIN = false>
struct Descent {
    using KF = KeyFmt<KB>;
    using K = typename KF::T;
    static constexpr bool WIDE = KB == 16;
    static constexpr int G = B / KPL;   // lanes per lookup in the cache-resident levels
    static constexpr int LPW = 64 / G;  // lookups per wavefront per round there
    // Hybrid mode (BIN with KPL < B): every lane owns R lookups and walks the
    // LDS-staged levels alone by binary search, then groups of G lanes take
    // the lookups over, one owner lane's at a time, for the lower levels.
    static constexpr bool kHybrid = BIN && KPL < B;
    static constexpr int kLS = leaf_slots_for(B, (int)sizeof(K));  // slots per leaf
    static constexpr int kLC = leaf_cap_for(B, (int)sizeof(K));    // keys (intervals) per leaf
    static constexpr int kLPER = kLS / G;                          // leaf slots per lane
    static constexpr uint64_t kStep = kHybrid ? 64ull * R : (uint64_t)LPW * R;  // lookups per wavefront step

    // Bytes of LDS the top levels of t take.
    static __host__ __device__ size_t lds_bytes(const TreeDesc& t) { return (size_t)t.lds_slots * sizeof(K); }

    // LDS slot permutation of the hybrid descent over 16-byte keys.  Its
    // lanes binary-search different nodes, probing the same slot of each:
    // with nodes laid out contiguously, that slot of every node falls in the
    // few banks a node's offset within a 256-byte row of the 64 four-byte
    // banks allows, and the wavefront's reads conflict.  So internal node n
    // keeps key k at slot k ^ lds_swz(n) of its LDS copy, lds_swz(n) taken
    // from the bits of n above those that place the node in its row.  At
    // b = 8 this took 128-bit key slots from 45.7 to 54.7 GLPS on the 200k
    // backbone FIB; with 8-byte keys (four 64-byte nodes per row) it cost
    // 1.7% on the same FIB, so narrower keys keep the plain layout.
    static constexpr bool kSwz = kHybrid && sizeof(K) == 16;
    static constexpr uint32_t kRowNodes = B * sizeof(K) >= 256 ? 1u : (uint32_t)(256 / (B * sizeof(K)));
    static __device__ __forceinline__ uint32_t lds_swz(uint32_t n)
    {
        if constexpr (kSwz)
            return (n / kRowNodes) & (uint32_t)(B - 1);
        else
            return 0;
    }

    // Copy the first t.lds_slots slots (the top t.lds_levels levels) to LDS,
    // internal nodes permuted by lds_swz, leaves (a whole tree in LDS) as they are.
    static __device__ void stage(const TreeDesc& t, uint4* lds_raw, int tid, int nthreads)
    {
        uint32_t done = 0;  // slots copied with the permutation
        if constexpr (kSwz) {
            done = t.lds_slots < t.leaf_base ? t.lds_slots : t.leaf_base;
            const K* src = static_cast<const K*>(t.keys);
            K* dst = reinterpret_cast<K*>(lds_raw);
            stage_items<4>(
                done, (uint32_t)tid, (uint32_t)nthreads, [&](uint32_t i) { return src[i]; },
                [&](uint32_t i, const K& v) {
                    const uint32_t n = i / (uint32_t)B, k = i % (uint32_t)B;
                    dst[n * (uint32_t)B + (k ^ lds_swz(n))] = v;
                });
        }
        // internal nodes are B * sizeof(K) >= 32 bytes: done is a whole number of 16-byte units
        const uint32_t first = (uint32_t)(done * sizeof(K) / 16);
        const uint32_t units = (uint32_t)(t.lds_slots * sizeof(K) / 16) - first;
        const uint4* src = static_cast<const uint4*>(t.keys) + first;
        uint4* dst = lds_raw + first;
        stage_items<4>(
            units, (uint32_t)tid, (uint32_t)nthreads, [&](uint32_t i) { return src[i]; },
            [&](uint32_t i, const uint4& v) { dst[i] = v; });
    }

    // The bottom internal level (level t.depth - 2) in LDS as the top 32 bits
    // of each of its keys, B - 1 per node (the sentinel slot is never
    // probed), after the t.lds_slots exact slots of the levels above: 4 bytes
    // per key instead of 8, so that this level fits beside them.
    static __device__ __forceinline__ uint32_t bottom_level(const TreeDesc& t) { return t.depth - 2; }
    static __device__ __forceinline__ uint32_t* bottom_tops(const void* lds, const TreeDesc& t)
    {
        return reinterpret_cast<uint32_t*>(const_cast<char*>(static_cast<const char*>(lds)) + (size_t)t.lds_slots * sizeof(K));
    }
    static __device__ void stage_bottom_tops(const TreeDesc& t, uint4* lds_raw, int tid, int nthreads)
    {
        static_assert(KB == 8 || KB == 16, "key tops are defined for 64- and 128-bit key slots");
        constexpr uint32_t W = KB / 4;  // 32-bit words per slot; word 1 is the top of the high word
        stage(t, lds_raw, tid, nthreads);
        if (t.depth < 2) return;
        const uint32_t lvl = bottom_level(t);
        const uint32_t keys = (t.off[lvl + 1] - t.off[lvl]) * (uint32_t)(B - 1);
        const uint32_t* src = static_cast<const uint32_t*>(t.keys);
        uint32_t* tops = bottom_tops(lds_raw, t);
        const uint32_t off = t.off[lvl];
        stage_items<16>(
            keys, (uint32_t)tid, (uint32_t)nthreads,
            [&](uint32_t i) {
                const uint32_t node = i / (uint32_t)(B - 1), s = i - node * (uint32_t)(B - 1);
                return src[(size_t)W * ((off + node) * (uint32_t)B + s) + 1];
            },
            [&](uint32_t i, uint32_t v) { tops[i] = v; });
    }

    // NW consecutive 32-bit words at p, with the widest loads their alignment
    // allows (p is aligned to NW * 4 bytes, or to 16 when NW is a multiple of 4).
    template <int NW>
    static __device__ __forceinline__ void load_words(const void* p, uint32_t* w)
    {
        if constexpr (NW % 4 == 0) {
            const uint4* q = static_cast<const uint4*>(p);
#pragma unroll
            for (int s = 0; s < NW / 4; ++s) {
                const uint4 v = q[s];
                w[4 * s] = v.x;
                w[4 * s + 1] = v.y;
                w[4 * s + 2] = v.z;
                w[4 * s + 3] = v.w;
            }
        } else if constexpr (NW % 2 == 0) {
            const uint2* q = static_cast<const uint2*>(p);
#pragma unroll
            for (int s = 0; s < NW / 2; ++s) {
                const uint2 v = q[s];
                w[2 * s] = v.x;
                w[2 * s + 1] = v.y;
            }
        } else {
            const uint32_t* q = static_cast<const uint32_t*>(p);
#pragma unroll
            for (int s = 0; s < NW; ++s) w[s] = q[s];
        }
    }

    // key s of a run of narrow keys held as words (KB 8: two words, KB 4: one) <= x
    static __device__ __forceinline__ int word_key_le(const uint32_t* w, int s, uint64_t xhi)
    {
        if constexpr (KB == 8)
            return (((uint64_t)w[2 * s + 1] << 32) | w[2 * s]) <= xhi;
        else
            return w[s] <= (uint32_t)(xhi >> 32);
    }

    // Keys <= x in the node whose first slot is keys[node0], summed over the
    // lookup's G lanes (lane j of the group is `j`).
    // Slot indexes of the global levels.  With 64-bit keys they are 32-bit
    // and address the array by a 32-bit byte offset from its (uniform) base:
    // the slot array stays below 4 GiB.  For the other widths the 64-bit
    // form measured faster.
    using SlotIdx = std::conditional_t<KB == 8, uint32_t, uint64_t>;
    static __device__ __forceinline__ const K* slot_ptr(const K* keys, SlotIdx slot)
    {
        if constexpr (KB != 8) return keys + slot;
        else return reinterpret_cast<const K*>(reinterpret_cast<const char*>(keys) + slot * (uint32_t)sizeof(K));
    }

    template <bool FROM_LDS>
    static __device__ __forceinline__ uint32_t node_count(const K* keys, SlotIdx node0, int j, uint64_t xhi,
                                                          uint64_t xlo)
    {
        if constexpr (BIN && FROM_LDS && KPL == B) {
            // one lane per lookup: branch-free binary search over the node's
            // slots.  It counts the keys <= x among slots 0..B-2 (B-1 at most):
            // the sentinel slot is never probed, which changes nothing because
            // only an address equal to the sentinel would count it, and that
            // address ends clamped on the last interval either way.
            uint32_t c = 0;
#pragma unroll
            for (int step = B / 2; step >= 1; step >>= 1) c += KF::le(keys[node0 + c + step - 1], xhi, xlo) ? step : 0;
            return c;
        }
        int cnt = 0;
        if constexpr (!WIDE && KPL * KB >= 8) {
            // narrow keys: each lane reads its KPL keys contiguously with
            // full-width loads, so a group covers its node with few loads
            constexpr int NW = KPL * KB / 4;
            uint32_t w[NW];
            load_words<NW>(slot_ptr(keys, node0 + (SlotIdx)(j * KPL)), w);
#pragma unroll
            for (int s = 0; s < KPL; ++s) cnt += word_key_le(w, s, xhi);
        } else {
            // 16-byte keys (or one 4-byte key per lane): key s*G + j, so one
            // load instruction covers G consecutive keys of each group's node
            const K* p = slot_ptr(keys, node0 + (SlotIdx)j);  // constant strides fold into the loads
#pragma unroll
            for (int s = 0; s < KPL; ++s) cnt += KF::le(p[s * G], xhi, xlo);
        }
        return (uint32_t)group_sum<G>(cnt);
    }

    // ---- leaf level.  A lookup's G lanes load the leaf's words (lane j of
    // the group is `j`: with kContig it holds slots [j*kLPER, (j+1)*kLPER),
    // else slots j, G + j, 2G + j, ...), count the keys <= x among them, and
    // turn the count into the interval index.  The interval's next hop sits
    // in the same leaf, so the lane that loaded it picks the word out of its
    // registers and the group reads it with one cross-lane shuffle.
    static constexpr int kb = (int)sizeof(K);
    static constexpr bool kContig = !WIDE && kLPER * kb >= 8;
    static constexpr int kW = kLPER * kb / 4;  // 32-bit words of a leaf per lane

    // lane of the group, and word of that lane, that hold byte `byte` of a leaf
    static __host__ __device__ constexpr uint32_t byte_lane(uint32_t byte)
    {
        return kContig ? byte / (kLPER * kb) : (byte / kb) % G;
    }
    static __host__ __device__ constexpr uint32_t byte_word(uint32_t byte)
    {
        return kContig ? (byte % (kLPER * kb)) / 4 : (byte / kb) / G * (kb / 4) + (byte % kb) / 4;
    }
    // which words of a lane can hold a next hop (the pick selects among them only)
    struct WordSet {
        bool v[kW];
    };
    static constexpr WordSet hop_words()
    {
        WordSet m{};
        for (int s = 0; s < kLC; ++s) m.v[byte_word(leaf_hop_byte(s, kb, kLC))] = true;
        return m;
    }
    static constexpr WordSet kHopWords = hop_words();

    struct LeafWords {
        uint32_t w[kW];
    };

    static __device__ __forceinline__ void leaf_load(const K* keys, SlotIdx node0, int j, LeafWords& L)
    {
        if constexpr (kContig) {
            load_words<kW>(slot_ptr(keys, node0 + (SlotIdx)(j * kLPER)), L.w);
        } else {
            const K* p = slot_ptr(keys, node0 + (SlotIdx)j);
#pragma unroll
            for (int s = 0; s < kLPER; ++s) {
                const K k = p[s * G];
                if constexpr (WIDE) {  // uint4: the key's four words in memory order
                    L.w[4 * s] = k.x;
                    L.w[4 * s + 1] = k.y;
                    L.w[4 * s + 2] = k.z;
                    L.w[4 * s + 3] = k.w;
                } else if constexpr (KB == 8) {
                    L.w[2 * s] = (uint32_t)k;
                    L.w[2 * s + 1] = (uint32_t)(k >> 32);
                } else {
                    L.w[s] = k;
                }
            }
        }
    }

    // keys <= x among the lane's key slots
    static __device__ __forceinline__ int leaf_lane_count(const LeafWords& L, int j, uint64_t xhi, uint64_t xlo)
    {
        int cnt = 0;
#pragma unroll
        for (int s = 0; s < kLPER; ++s) {
            const uint32_t slot = kContig ? (uint32_t)(j * kLPER + s) : (uint32_t)(s * G + j);
            int le;
            if constexpr (WIDE)
                le = KF::le(make_uint4(L.w[4 * s], L.w[4 * s + 1], L.w[4 * s + 2], L.w[4 * s + 3]), xhi, xlo);
            else
                le = word_key_le(L.w, s, xhi);
            cnt += leaf_slot_is_key(slot, kb, kLC) ? le : 0;
        }
        return cnt;
    }

    // interval index of a count c of keys <= x in leaf q (c >= 1: interval 0
    // starts at 0); indexes fit 32 bits (a FIB has fewer than 2^31 intervals)
    static __device__ __forceinline__ uint32_t leaf_index(const TreeDesc& t, uint32_t q, uint32_t c)
    {
        const uint32_t idx = q * (uint32_t)kLC + c - 1, last = (uint32_t)t.m_minus_1;
        return idx < last ? idx : last;
    }

    // next hop of the leaf's interval `pos`, read by every lane of the group
    // (lane0 is the group's first lane)
    static __device__ __forceinline__ uint16_t leaf_pick_hop(const LeafWords& L, uint32_t pos, int lane0)
    {
        const uint32_t byte = leaf_hop_byte(pos, kb, kLC);
        const uint32_t word = byte_word(byte);
        uint32_t sel = 0;
#pragma unroll
        for (int k = 0; k < kW; ++k)
            if (kHopWords.v[k]) sel = word == (uint32_t)k ? L.w[k] : sel;
        if constexpr (G > 1) sel = (uint32_t)__shfl((int)sel, lane0 + (int)byte_lane(byte), 64);
        return (uint16_t)(sel >> (8 * (byte & 2)));
    }

    // Each lane holds exactly one block of the blocked leaf format (64-bit
    // keys, 32 bytes per lane): its keys and their next hops.  (With 32-bit
    // keys the same pick measured slower than the generic one, and is off.)
    static constexpr bool kBlockLane = kContig && kLPER * kb == 32 && kb == 8;
    static constexpr uint32_t kBlockKeys = kb == 8 ? 3 : 5;   // keys per block
    static constexpr uint32_t kBlockHop0 = kb == 8 ? 24 : 20;  // byte of the block's first next hop

    // Next hop (low 16 bits) of the lane's own block for its key cl - 1, cl in
    // 1..kBlockKeys (cl = 0 gives an unused value).  A byte permute of the
    // word pair holding the hops takes bytes 2(cl-1) and 2(cl-1)+1 of it and
    // zeroes the rest; with 32-bit keys the fifth hop is in the next word.
    static __device__ __forceinline__ uint32_t block_hop(const LeafWords& L, uint32_t cl)
    {
        constexpr int w0 = kBlockHop0 / 4;
        const uint32_t pick = __builtin_amdgcn_perm(L.w[w0 + 1], L.w[w0], cl * 0x202u + (0x0c0c0100u - 0x202u));
        if constexpr (kb == 8) return pick;
        else return cl == 5 ? L.w[w0 + 2] : pick;
    }

    // Whether x is all ones in the key width: it then counts the sentinel
    // padding of the last leaf too, and its interval is the last one.
    static __device__ __forceinline__ bool key_all_ones(uint64_t xhi, uint64_t xlo)
    {
        if constexpr (KB == 16) return (xhi & xlo) == ~0ull;
        else if constexpr (KB == 8) return xhi == ~0ull;
        else return (uint32_t)(xhi >> 32) == ~0u;
    }

    // NR lookups' leaves by lane groups: all loads first, then the searches.
    template <int NR>
    static __device__ __forceinline__ void leaf_groups(const TreeDesc& t, const K* keys, const uint32_t* q,
                                                       const uint64_t* xh, const uint64_t* xl, int j, int lane0,
                                                       uint32_t* idx, uint16_t* hop, uint32_t* cnt)
    {
        LeafWords L[NR];
#pragma unroll
        for (int u = 0; u < NR; ++u) leaf_load(keys, t.leaf_base + (SlotIdx)q[u] * kLS, j, L[u]);
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const uint32_t c = (uint32_t)group_sum<G>(leaf_lane_count(L[u], j, xh[u], xl[u]));
            cnt[u] = c;
            idx[u] = leaf_index(t, q[u], c);
            hop[u] = leaf_pick_hop(L[u], idx[u] - q[u] * (uint32_t)kLC, lane0);
        }
    }
    template <int NR>
    static __device__ __forceinline__ void leaf_groups(const TreeDesc& t, const K* keys, const uint32_t* q,
                                                       const uint64_t* xh, const uint64_t* xl, int j, int lane0,
                                                       uint32_t* idx, uint16_t* hop)
    {
        uint32_t cnt[NR];
        leaf_groups<NR>(t, keys, q, xh, xl, j, lane0, idx, hop, cnt);
    }

    // The same when every lane holds one block (kBlockLane); res[u] is the
    // interval index (index_out) or the next hop.
    template <int NR>
    static __device__ __forceinline__ void leaf_blocks(const TreeDesc& t, const K* keys, const uint32_t* q,
                                                       const uint64_t* xh, const uint64_t* xl, int j, int lane0,
                                                       int index_out, uint32_t* res, uint32_t* cnt)
    {
        LeafWords L[NR];
#pragma unroll
        for (int u = 0; u < NR; ++u) leaf_load(keys, t.leaf_base + (SlotIdx)q[u] * kLS, j, L[u]);
        // The keys <= x are a prefix of the leaf's keys (unless x is all ones
        // in the key width): the lanes before the last one holding such a key
        // have all of theirs <= x, so that lane is the count of lanes with any,
        // minus one, and its own count picks the hop in its block.  One group
        // sum adds both counts: keys in the low byte, lanes above it.
        const uint32_t last_hop = t.last_hop;
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const uint32_t cl = (uint32_t)leaf_lane_count(L[u], j, xh[u], xl[u]);
            const uint32_t sum = (uint32_t)group_sum<G>((int)(cl + (min(cl, 1u) << 8)));
            const uint32_t lanes = sum >> 8;  // >= 1: the leaf's first key is <= x
            // the upper 16 bits of the hop are not part of it (hops are uint16)
            const uint32_t got =
                (uint32_t)__builtin_amdgcn_ds_bpermute((lane0 + (int)lanes - 1) << 2, (int)block_hop(L[u], cl));
            const uint32_t hop = key_all_ones(xh[u], xl[u]) ? last_hop : got;
            res[u] = index_out ? leaf_index(t, q[u], sum & 0xFFu) : hop;
            cnt[u] = sum & 0xFFu;
        }
    }
    template <int NR>
    static __device__ __forceinline__ void leaf_blocks(const TreeDesc& t, const K* keys, const uint32_t* q,
                                                       const uint64_t* xh, const uint64_t* xl, int j, int lane0,
                                                       int index_out, uint32_t* res)
    {
        uint32_t cnt[NR];
        leaf_blocks<NR>(t, keys, q, xh, xl, j, lane0, index_out, res, cnt);
    }

    // One lane, leaf in LDS: the count by branch-free binary search over the
    // leaf's keys, and the next hop read directly.
    static __device__ __forceinline__ void leaf_lane(const TreeDesc& t, const K* keys, uint32_t q, uint64_t xhi,
                                                     uint64_t xlo, uint32_t* idx, uint16_t* hop)
    {
        const size_t node0 = t.leaf_base + (size_t)q * kLS;
        uint32_t c = 0;
#pragma unroll
        for (int step = kLS / 2; step >= 1; step >>= 1) {
            const uint32_t probe = c + step - 1;
            c += (probe < (uint32_t)kLC && KF::le(keys[node0 + leaf_key_slot(probe, kb)], xhi, xlo)) ? step : 0;
        }
        *idx = leaf_index(t, q, c);
        const uint8_t* leaf = reinterpret_cast<const uint8_t*>(keys + node0);
        *hop = *reinterpret_cast<const uint16_t*>(leaf + leaf_hop_byte(*idx - q * (uint32_t)kLC, kb, kLC));
    }

    template <bool FROM_LDS>
    static __device__ __forceinline__ uint32_t lane_bincount(const K* keys, size_t node0, uint64_t xhi, uint64_t xlo)
    {
        // from LDS, 16-byte keys are permuted within the node (stage)
        const uint32_t sw = FROM_LDS ? lds_swz((uint32_t)(node0 / B)) : 0u;
        uint32_t c = 0;  // keys <= x among slots 0..B-2 (see node_count)
#pragma unroll
        for (int step = B / 2; step >= 1; step >>= 1)
            c += KF::le(keys[node0 + ((c + (uint32_t)step - 1) ^ sw)], xhi, xlo) ? step : 0;
        return c;
    }

    // The bottom internal level from its key tops, one lane per lookup: a
    // binary search counts the tops <= x's top half (exact on the tops).  The
    // keys it counts whose top equals x's are the end of that prefix, and the
    // ones among them above x are a suffix of it, so a lane whose last counted
    // top ties walks back over them, one whole key read from device memory
    // per step (one step, nearly always).  bottom_search issues the first of
    // those reads; bottom_finish, called after the lane hand-off's address
    // shuffles, uses it, so that its round trip overlaps them.
    struct Bottom {
        uint32_t c[R], last[R];
        K tk[R];  // the key c - 1, read when its top ties
    };
    // key > x for a whole key read from device memory
    static __device__ __forceinline__ bool key_gt(const K& k, uint64_t xh, uint64_t xl) { return !KF::le(k, xh, xl); }
    static __device__ __forceinline__ void bottom_search(const TreeDesc& t, const uint32_t* tops, const uint64_t* xh,
                                                         const uint32_t* q, Bottom& bs)
    {
        const uint32_t lvl = bottom_level(t), lim = t.last[lvl + 1];
        const K* gkeys = static_cast<const K*>(t.keys);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t tx = (uint32_t)(xh[r] >> 32), n0 = q[r] * (uint32_t)(B - 1);
            uint32_t c = 0, last = 0;
#pragma unroll
            for (int step = B / 2; step >= 1; step >>= 1) {
                const uint32_t v = tops[n0 + c + (uint32_t)(step - 1)];
                const bool le = v <= tx;
                last = le ? v : last;
                c += le ? (uint32_t)step : 0u;
            }
            bs.c[r] = c;
            bs.last[r] = last;
            // Key c - 1 of node q separates leaves qB + c - 1 and qB + c, and is
            // the first key of leaf qB + c, whose slot 0 holds it too.  Reading it
            // there keeps the bottom level out of the caches, and when the tie
            // resolves to "<=" that leaf is the one read next.  Past the last leaf
            // the separator is the sentinel; the last leaf's first key then gives
            // the same child once clamped to the last leaf (if it is <= x, both
            // end at the last leaf; if > x, both step back).  Every lane loads;
            // the untied ones all read slot 0 (one shared line), so the load is
            // not in a branch and its wait can follow the shuffles.
            const bool tie = c > 0 && last == tx;
            const uint32_t leaf = min(q[r] * (uint32_t)B + c, lim);
            bs.tk[r] = *slot_ptr(gkeys, tie ? (SlotIdx)t.leaf_base + (SlotIdx)leaf * (SlotIdx)kLS : (SlotIdx)0);
        }
    }
    static __device__ __forceinline__ void bottom_finish(const TreeDesc& t, const uint32_t* tops, const uint64_t* xh,
                                                         const uint64_t* xl, uint32_t* q, const Bottom& bs)
    {
        const uint32_t lvl = bottom_level(t), lim = t.last[lvl + 1];
        const K* gkeys = static_cast<const K*>(t.keys);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t tx = (uint32_t)(xh[r] >> 32), n0 = q[r] * (uint32_t)(B - 1);
            uint32_t c = bs.c[r];
            if (c > 0 && bs.last[r] == tx && key_gt(bs.tk[r], xh[r], xl[r])) {
                --c;  // further steps read key c - 1 from its leaf's slot 0 as well
                while (c > 0 && tops[n0 + c - 1] == tx &&
                       key_gt(*slot_ptr(gkeys, (SlotIdx)t.leaf_base + (SlotIdx)min(q[r] * (uint32_t)B + c, lim) *
                                                                          (SlotIdx)kLS),
                              xh[r], xl[r]))
                    --c;
            }
            q[r] = min(q[r] * B + c, lim);
        }
    }

    static __device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
    {
        const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
        return ((uint64_t)hi << 32) | lo;
    }

    static __device__ __forceinline__ void store(void* out, int index_out, uint64_t i, uint32_t idx, uint16_t hop)
    {
        if (index_out)
            __builtin_nontemporal_store(idx, static_cast<uint32_t*>(out) + i);
        else
            __builtin_nontemporal_store(hop, static_cast<uint16_t*>(out) + i);
    }

    // Address i of a batch: 16-byte {hi, lo} records, or 4-byte IPv4
    // addresses, which stand for the 128-bit address with those 32 bits on top.
    static __device__ __forceinline__ void fetch(const u64x2* a, uint64_t i, uint64_t& hi, uint64_t& lo)
    {
        const u64x2 v = __builtin_nontemporal_load(a + i);
        hi = v.x;
        lo = v.y;
    }
    static __device__ __forceinline__ void fetch(const uint32_t* a, uint64_t i, uint64_t& hi, uint64_t& lo)
    {
        hi = (uint64_t)__builtin_nontemporal_load(a + i) << 32;
        lo = 0;
    }

    // TOPS: lds holds the exact levels above the bottom internal one, then
    // that level's key tops (stage_bottom_tops); else the first t.lds_levels
    // levels' keys (stage).
    template <typename A, bool TOPS = false>
    static __device__ __forceinline__ void step_hybrid(const TreeDesc& t, const void* lds, const A* addrs,
                                                       uint64_t base, uint64_t n, void* out, int index_out)
    {
        const K* lds_keys = static_cast<const K*>(lds);  // with TOPS: the exact levels above the bottom one
        const int lane = threadIdx.x & 63;
        uint64_t xh[R], xl[R];
        uint32_t q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = base + (uint64_t)r * 64 + lane;
            fetch(addrs, i < n ? i : n - 1, xh[r], xl[r]);
            q[r] = 0;
        }
        // LDS-staged levels, one lane per lookup
        uint32_t lds_internal = t.lds_levels < t.depth - 1 ? t.lds_levels : t.depth - 1;
        for (uint32_t l = 0; l < lds_internal; ++l) {
            const uint32_t off = t.off[l], lim = t.last[l + 1];
#pragma unroll
            for (int r = 0; r < R; ++r)
                q[r] = min(q[r] * B + lane_bincount<true>(lds_keys, (size_t)(off + q[r]) * B, xh[r], xl[r]), lim);
        }
        Bottom bs;
        if constexpr (TOPS) {  // lds_levels = depth - 2: the bottom internal level from its tops
            if (t.depth >= 2) {
                bottom_search(t, bottom_tops(lds, t), xh, q, bs);
                lds_internal = t.depth - 1;
            }
        }
        if (!TOPS && t.lds_levels >= t.depth) {  // the whole tree is in LDS
#pragma unroll
            for (int r = 0; r < R; ++r) {
                uint32_t idx;
                uint16_t hop;
                leaf_lane(t, lds_keys, q[r], xh[r], xl[r], &idx, &hop);
                const uint64_t i = base + (uint64_t)r * 64 + lane;
                if (i < n) store(out, index_out, i, idx, hop);
            }
            return;
        }
        // lower levels: G lanes per lookup; round u serves owner lane
        // (u % G) * LPW + lane / G, its lookup u / G
        constexpr int T = R * G;
        const int grp = lane / G, j = lane % G;
        const K* gkeys = static_cast<const K*>(t.keys);
        uint64_t yh[T], yl[T];
        uint32_t p[T];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const int owner = (u % G) * LPW + grp;
            yh[u] = shfl64(xh[u / G], owner);
            yl[u] = WIDE ? shfl64(xl[u / G], owner) : 0;
        }
        if constexpr (TOPS) {  // the tie reads were issued before the shuffles above
            // Keep the first use of those reads (and so the wait for them)
            // after the shuffles: the compiler would otherwise hoist the
            // comparison, and the wait, above them.  The empty asm only marks
            // the values as changed here; it reads and writes no memory.
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (WIDE) asm volatile("" : "+v"(bs.tk[r].x), "+v"(bs.tk[r].y), "+v"(bs.tk[r].z), "+v"(bs.tk[r].w));
                else asm volatile("" : "+v"(bs.tk[r]));
            }
            if (t.depth >= 2) bottom_finish(t, bottom_tops(lds, t), xh, xl, q, bs);
        }
#pragma unroll
        for (int u = 0; u < T; ++u) p[u] = (uint32_t)__shfl((int)q[u / G], (u % G) * LPW + grp, 64);
        for (uint32_t l = lds_internal; l + 1 < t.depth; ++l) {
            const uint32_t off = t.off[l], lim = t.last[l + 1];
#pragma unroll
            for (int u = 0; u < T; ++u)
                p[u] = min(p[u] * B + node_count<false>(gkeys, (SlotIdx)(off + p[u]) * B, j, yh[u], yl[u]), lim);
        }
        uint32_t res[T];
        if constexpr (kBlockLane) {
            leaf_blocks<T>(t, gkeys, p, yh, yl, j, lane - j, index_out, res);
        } else {
            uint32_t idx[T];
            uint16_t hop[T];
            leaf_groups<T>(t, gkeys, p, yh, yl, j, lane - j, idx, hop);
#pragma unroll
            for (int u = 0; u < T; ++u) res[u] = index_out ? idx[u] : hop[u];
        }
        // hand every result back to the lane that owns its lookup, so each of
        // the R stores writes 64 consecutive results: owner lane L's lookup r
        // was round r*G + L/LPW, computed by group L%LPW
        const int g = lane / LPW, src = (lane % LPW) * G;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t v = 0;
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const uint32_t got = (uint32_t)__shfl((int)res[r * G + k], src, 64);
                v = k == g ? got : v;
            }
            const uint64_t i = base + (uint64_t)r * 64 + lane;
            if (i < n) store(out, index_out, i, v, (uint16_t)v);
        }
    }

    // Lookups [base, base + kStep) of a batch of n >= 1 addresses.  Every lane
    // of the wavefront must call this together (DPP crosses lanes).
    template <typename A>
    static __device__ __forceinline__ void step(const TreeDesc& t, const K* lds_keys, const A* addrs,
                                                uint64_t base, uint64_t n, void* out, int index_out)
    {
        if constexpr (kHybrid) {
            step_hybrid(t, lds_keys, addrs, base, n, out, index_out);
            return;
        }
        const int lane = threadIdx.x & 63;
        const int grp = lane / G;
        const int j = lane % G;
        const K* gkeys = static_cast<const K*>(t.keys);
        uint64_t xhi[R], xlo[R];
        uint32_t q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = base + (uint64_t)r * LPW + grp;
            fetch(addrs, i < n ? i : n - 1, xhi[r], xlo[r]);
            q[r] = 0;
        }
        for (uint32_t l = 0; l + 1 < t.depth; ++l) {
            const uint32_t off = t.off[l], lim = t.last[l + 1];
            if (l < t.lds_levels) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    q[r] = min(q[r] * B + node_count<true>(lds_keys, (SlotIdx)(off + q[r]) * B, j, xhi[r], xlo[r]), lim);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    q[r] = min(q[r] * B + node_count<false>(gkeys, (SlotIdx)(off + q[r]) * B, j, xhi[r], xlo[r]), lim);
            }
        }
        if constexpr (kBlockLane) {
            uint32_t res[R];
            if (t.lds_levels < t.depth)
                leaf_blocks<R>(t, gkeys, q, xhi, xlo, j, lane - j, index_out, res);
            else
                leaf_blocks<R>(t, lds_keys, q, xhi, xlo, j, lane - j, index_out, res);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t i = base + (uint64_t)r * LPW + grp;
                if (j == 0 && i < n) store(out, index_out, i, res[r], (uint16_t)res[r]);
            }
            return;
        }
        uint32_t idx[R];
        uint16_t hop[R];
        if (t.lds_levels < t.depth) {
            leaf_groups<R>(t, gkeys, q, xhi, xlo, j, lane - j, idx, hop);
        } else if constexpr (BIN && KPL == B) {
#pragma unroll
            for (int r = 0; r < R; ++r) leaf_lane(t, lds_keys, q[r], xhi[r], xlo[r], &idx[r], &hop[r]);
        } else {
            leaf_groups<R>(t, lds_keys, q, xhi, xlo, j, lane - j, idx, hop);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = base + (uint64_t)r * LPW + grp;
            if (j == 0 && i < n) store(out, index_out, i, idx[r], hop[r]);
        }
    }
};

// Key i of the dense interval order, read from the leaf level of the tree.
template <int B, int KB>
__device__ inline typename KeyFmt<KB>::T leaf_key(const TreeDesc& t, uint64_t i)
{
    constexpr int kb = KB;
    constexpr uint64_t LC = leaf_cap_for(B, kb), LS = leaf_slots_for(B, kb);
    const auto* keys = static_cast<const typename KeyFmt<KB>::T*>(t.keys);
    return keys[t.leaf_base + (i / LC) * LS + leaf_key_slot((uint32_t)(i % LC), kb)];
}

// Picks KernelOf<B, KPL, R, KB, BS, BIN>::get() for runtime values among the
// compiled-in variants: B in {8, 16, 32}, KPL in {1, 2, 4, 8, 16} with B/KPL
// in [1, 32], R in {1, 2, 4}, KB (key slot bytes) in {4, 8, 16}, BS in
// {512, 1024}, and BIN (binary search by one lane per lookup in the LDS
// levels; with KPL < B the lower levels are then shared by B/KPL lanes, for
// B/KPL in {2, 4}).
template <template <int, int, int, int, int, bool> class KernelOf>
struct VariantTable {
    using Fn = typename KernelOf<8, 1, 1, 16, 512, false>::Fn;

    template <int B, int KPL, int KB, int BS, bool BIN>
    static Fn by_r(int R)
    {
        switch (R) {
        case 1: return KernelOf<B, KPL, 1, KB, BS, BIN>::get();
        case 2: return KernelOf<B, KPL, 2, KB, BS, BIN>::get();
        case 4: return KernelOf<B, KPL, 4, KB, BS, BIN>::get();
        default: return nullptr;
        }
    }
    template <int B, int KB, int BS>
    static Fn by_kpl(int kpl, int R, bool bin)
    {
        if (bin) {
            if (kpl == B) return by_r<B, B, KB, BS, true>(R);
            if (kpl == B / 2) return by_r<B, B / 2, KB, BS, true>(R);
            if (kpl == B / 4) return by_r<B, B / 4, KB, BS, true>(R);
            return nullptr;
        }
        switch (kpl) {
        case 1: return by_r<B, 1, KB, BS, false>(R);
        case 2: return by_r<B, 2, KB, BS, false>(R);
        case 4: return by_r<B, 4, KB, BS, false>(R);
        case 8: return by_r<B, 8, KB, BS, false>(R);
        case 16: if constexpr (B >= 16) return by_r<B, 16, KB, BS, false>(R); else return nullptr;
        default: return nullptr;
        }
    }
    template <int KB, int BS>
    static Fn by_b(int B, int kpl, int R, bool bin)
    {
        switch (B) {
        case 8: return by_kpl<8, KB, BS>(kpl, R, bin);
        case 16: return by_kpl<16, KB, BS>(kpl, R, bin);
        case 32: return by_kpl<32, KB, BS>(kpl, R, bin);
        default: return nullptr;
        }
    }
    template <int BS>
    static Fn by_kb(int B, int kpl, int R, int kb, bool bin)
    {
        switch (kb) {
        case 4: return by_b<4, BS>(B, kpl, R, bin);
        case 8: return by_b<8, BS>(B, kpl, R, bin);
        case 16: return by_b<16, BS>(B, kpl, R, bin);
        default: return nullptr;
        }
    }
    static Fn pick(int B, int kpl, int R, int kb, int bs, bool bin = false)
    {
        if (bs == 512) return by_kb<512>(B, kpl, R, kb, bin);
        if (bs == 1024) return by_kb<1024>(B, kpl, R, kb, bin);
        return nullptr;
    }
};

}  // namespace planb
