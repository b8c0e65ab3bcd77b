/*
 * planb.h -- C ABI of an MI355X (gfx950) library for batched IPv6
 * longest-prefix-match lookup on a linearized B+-tree of elementary intervals.
 *
 * Method: "PlanB: Efficient Software IPv6 Lookup with Linearized B+-Tree"
 * (arXiv 2604.14650).  Section references below are to that paper.
 *
 * Conventions shared by every entry point
 *  - An IPv6 address or prefix is a planb_addr_t {hi, lo}: hi holds address
 *    bytes 0..7 read as a big-endian integer, lo bytes 8..15.  In memory it is
 *    two little-endian uint64 words, hi first: 16 bytes.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are GPU memory
 *    of the current HIP device (hipMalloc, or a torch CUDA tensor).
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Lookup calls only enqueue work: results are valid after the stream is
 *    synchronised.  They never synchronise, and none allocates except
 *    planb_lookup_learned, which takes its fallback queue from the
 *    stream-ordered pool (planb_lookup_learned_noalloc allocates nothing).
 *  - Functions returning int give PLANB_OK (0) or a negative planb_status;
 *    functions returning a pointer give NULL on failure.  On failure
 *    planb_last_error() returns a message for the calling thread.
 */
#ifndef PLANB_H
#define PLANB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct planb_addr {
    uint64_t hi; /* address bits 127..64 */
    uint64_t lo; /* address bits 63..0  */
} planb_addr_t;

/* The next hop returned for an address no rule covers (no ::/0 in the FIB).
 * It stands for the paper's "-1" of Algorithm 2 / the default route of the
 * interval-partitioning step; it is reserved and may not be a rule's next hop. */
#define PLANB_NO_ROUTE 0xFFFFu

typedef enum planb_status {
    PLANB_OK = 0,
    PLANB_EINVAL = -1,  /* bad argument: length > 128, reserved next hop, NULL or misaligned pointer */
    PLANB_EDUP = -2,    /* the same (prefix, length) given twice after masking host bits */
    PLANB_ENOMEM = -3,  /* host or device allocation failed */
    PLANB_EDEVICE = -4, /* a HIP call or kernel launch failed */
    PLANB_ERANGE = -5   /* a size exceeds what the structure or call supports */
} planb_status_t;

/* Opaque handle of one built FIB: owns the device copies of the key array
 * (the linearized B+-tree) and of the next-hop array, plus any learned model. */
typedef struct planb_fib planb_fib_t;

/* Build-time parameters.  Zero-initialise and set what you need. */
typedef struct planb_params {
    uint32_t fanout;        /* b: children per internal node, 8, 16 or 32 (0 -> 16).
                               A node holds k = b-1 keys plus one sentinel slot:
                               b key slots per node. */
    uint32_t keys_per_lane; /* initial lookup tuning, see planb_tuning_t (0 -> default) */
    int32_t lds_levels;     /* initial lookup tuning, see planb_tuning_t (0 -> default) */
    uint32_t flags;         /* PLANB_FLAG_* */
    uint32_t key_bits;      /* stored key width: 0 = automatic, 128 = always the full
                               16-byte key, 64 = only the high 64 bits (8-byte slots),
                               32 = only the top 32 bits (4-byte slots).
                               64 is exact exactly when every interval start has a
                               zero low word -- e.g. when no prefix is longer than /64
                               (the paper's own key width, Section 3 "Parameter
                               Tuning"); 32 exactly when every start's low 96 bits are
                               zero -- e.g. IPv4 rules placed in the top 32 bits
                               (planb_lookup_v4).  Automatic picks the narrowest exact
                               width; asking for an inexact one fails with
                               PLANB_EINVAL. */
} planb_params_t;

/* Merge neighbouring elementary intervals that resolve to the same next hop.
 * Off by default: the paper does not merge; merging changes no result. */
#define PLANB_FLAG_MERGE_EQUAL_NH 1u

/*
 * planb_build -- the pre-computation of Section 3 ("From 2D Prefixes to 1D
 * Intervals", "1D Search with Linearized B+-Tree", Algorithm 2), on the host,
 * then one upload to the device.
 *   prefixes  host, n records; host bits beyond each length are ignored (masked)
 *   lengths   host, n prefix lengths 0..128
 *   next_hops host, n values 0..0xFFFE (0xFFFF is PLANB_NO_ROUTE and rejected)
 *   n         may be 0: every lookup then returns PLANB_NO_ROUTE
 * Steps: mask; range conversion [P, P + 2^(128-L)) in 129-bit arithmetic (an
 * end of 2^128 produces no boundary); sort the 2n boundary events (address,
 * END before START, START by ascending length); one sweep with a stack of next
 * hops yields the elementary intervals (an interval at address 0 always exists,
 * with ::/0's next hop or PLANB_NO_ROUTE); the interval starts fill the leaves
 * of a fanout-b tree whose internal separators are the minima of the child
 * subtrees.  The inputs are copied; the caller keeps ownership.
 * Errors: NULL with PLANB_EINVAL (length > 128, next hop 0xFFFF, NULL array
 * with n > 0), PLANB_EDUP, PLANB_ENOMEM, PLANB_EDEVICE, PLANB_ERANGE (2^31 or
 * more intervals, or a slot array of 4 GiB or more: the kernels address it
 * with 32-bit byte offsets).
 */
planb_fib_t* planb_build(const planb_addr_t* prefixes, const uint8_t* lengths,
                         const uint16_t* next_hops, size_t n);

/*
 * The same build run on the device (Section 3.6 rebuilds the structure from
 * the rule set on every update; this keeps that rebuild next to the lookups).
 * prefixes (16-byte aligned), lengths and next_hops are DEVICE arrays of n
 * rules; params as for planb_build_ex; the work runs on `stream` and the call
 * returns when the FIB is ready (it synchronises the stream twice, to size the
 * tree and to copy the intervals back for planb_export_intervals and
 * training).  The result -- intervals, tree image, next hops, errors -- is the
 * one planb_build_ex gives for the same rules.  At most 2^30 - 1 rules.
 */
planb_fib_t* planb_build_device(const planb_addr_t* prefixes, const uint8_t* lengths, const uint16_t* next_hops,
                                size_t n, const planb_params_t* params, void* stream);
planb_fib_t* planb_build_ex(const planb_addr_t* prefixes, const uint8_t* lengths,
                            const uint16_t* next_hops, size_t n, const planb_params_t* params);

/*
 * planb_lookup -- batched search of Algorithm 1 / Listing 1 (Section 3, "Search
 * on Linearized B+-Tree", "Vectorization", "Batching", "Branch-Free Traversal")
 * on the GPU.  For each address x, descends the tree: at every level the node's
 * keys <= x are counted and the count selects the child; at the leaf the count
 * gives the predecessor interval, whose next hop is written.
 *   addrs  device, n records, 16-byte aligned
 *   out    device, n uint16 next hops, 2-byte aligned
 *   n      0 is a no-op; must be < 2^40
 * Returns PLANB_OK, PLANB_EINVAL (NULL fib / NULL or misaligned pointer with
 * n > 0), PLANB_ERANGE, PLANB_EDEVICE (launch failed).
 */
int planb_lookup(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n,
                 uint16_t* out, void* stream);

/* Same descent, but writes the index (0..m-1) of the elementary interval that
 * holds each address instead of its next hop.  out: device, n uint32. */
int planb_lookup_index(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n,
                       uint32_t* out, void* stream);

/* Releases the handle (Section 3, "Dynamic FIB Update": the replaced
 * structure is freed once the lookups in flight on it complete).  Every call
 * that enqueues work reading a FIB -- the lookup, batch, graph, learned,
 * model and table-set calls -- records an event after that work on its
 * stream.  planb_free returns at once: the device memory is freed in stream
 * order behind those events, on a library stream, so neither the host nor any
 * other stream waits.  Work captured into a caller's own graph is not
 * recorded; keep the FIB until that graph's last replay has completed.  The
 * handle may not be used after the call.  NULL is ignored. */
void planb_free(planb_fib_t* fib);

/* Message describing the last failure on the calling thread ("" if none). */
const char* planb_last_error(void);

/* planb_status of the last failure on the calling thread (0 if none); useful
 * after a call that returns NULL.  Reset by planb_build* calls. */
int planb_last_status(void);

/*
 * IPv4: planb_lookup over n 4-byte addresses (device, 4-byte aligned), each
 * standing for the 128-bit address with those 32 bits on top, for a FIB built
 * from rules of at most /32 placed the same way (so its keys are 32-bit;
 * PLANB_EINVAL otherwise).  The same kernel with 4-byte key slots and 4-byte
 * address loads: 6 bytes of HBM traffic per lookup instead of 18.
 */
int planb_lookup_v4(const planb_fib_t* fib, const uint32_t* addrs, size_t n, uint16_t* out, void* stream);

/*
 * The same answers as planb_lookup by plain binary search over the sorted
 * interval starts, one lane per address, then a read of the next-hop array:
 * the GPU analogue of the std::lower_bound baseline of the paper's ablation
 * (Section 4), for comparing the tree against it.  Arguments and errors as
 * planb_lookup.
 */
int planb_lookup_bsearch(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint16_t* out, void* stream);

/* m, the number of elementary intervals (Section 3: at most 2n + 1). */
size_t planb_num_intervals(const planb_fib_t* fib);

/* Copies min(m, cap) interval starts and next hops to host memory and returns
 * how many were written (or a negative status).  Either array may be NULL. */
long long planb_export_intervals(const planb_fib_t* fib, planb_addr_t* starts,
                                 uint16_t* next_hops, size_t cap);

/* Copies the FIB's device slot array (the image planb_build_image describes)
 * to host memory and returns its size in bytes, or only returns the size when
 * image is NULL or cap_bytes is too small; negative status on error.
 * Synchronous. */
long long planb_export_image(const planb_fib_t* fib, void* image, size_t cap_bytes);

#define PLANB_MAX_LEVELS 16

/*
 * Shape of a built tree.  Internal nodes have `slots` key slots (b - 1 keys
 * and a sentinel) and are counted and offset in nodes.  Leaves follow them in
 * the same slot array from slot leaf_base on, each leaf_slots slots long and
 * holding leaf_keys interval starts (interval i in leaf i / leaf_keys).  In a
 * built FIB a leaf also carries the next hops of its intervals: leaf_keys
 * uint16 values beside its keys, so that a lookup reads its answer from the
 * line it already loaded: with 128-bit slots right after the keys (byte
 * leaf_keys * 16 of the leaf); with 64-bit slots in 32-byte blocks of three
 * keys and their three hops; with 32-bit slots in 32-byte blocks of five keys
 * and their five hops.
 * A FIB's leaf is max(b slots, 128 bytes) long and leaf_keys is the number
 * of (key, next hop) pairs that fit; in the paper's layout (planb_layout)
 * leaves are ordinary nodes: leaf_keys = b - 1, leaf_slots = slots.
 */
typedef struct planb_info {
    uint64_t intervals;                 /* m */
    uint32_t fanout;                    /* b */
    uint32_t slots;                     /* key slots per internal node (b: k keys + 1 sentinel) */
    uint32_t depth;                     /* D: levels including the leaf level */
    uint32_t key_bits;                  /* 128, 64 or 32, see planb_params_t */
    uint64_t level_nodes[PLANB_MAX_LEVELS];      /* allocated nodes per level (leaves last) */
    uint64_t level_offset[PLANB_MAX_LEVELS + 1]; /* first node of each level (internal levels) */
    uint64_t key_bytes;                 /* device bytes of the slot array (keys + in-leaf next hops) */
    uint64_t value_bytes;               /* device bytes of the plain next-hop array */
    uint32_t leaf_keys;                 /* interval starts per leaf */
    uint32_t leaf_slots;                /* slots per leaf */
    uint64_t leaf_base;                 /* slot index of leaf 0 */
} planb_info_t;

int planb_get_info(const planb_fib_t* fib, planb_info_t* info);

/*
 * Launch shape of the lookup kernels for one built FIB (changes no result):
 *   keys_per_lane      each lane compares this many keys of a node, so
 *                      b / keys_per_lane lanes of a wavefront cooperate on one
 *                      lookup; a power of two dividing b, b/keys_per_lane <= 32
 *   lds_levels         how many top levels each workgroup stages in LDS
 *                      (0..depth; -1 = the deepest that fits 64 KiB)
 *   lookups_per_group  independent lookups each lane group keeps in flight (1, 2 or 4)
 *   block_threads      workgroup size, 512 or 1024
 *   lds_search         0: every lane compares all its keys of a node;
 *                      1: in the LDS-staged levels every lane walks its own
 *                      lookups by binary search inside the nodes; the lower
 *                      levels are then shared by fanout/keys_per_lane lanes
 *                      (1, 2 or 4), which take the lookups over by shuffles;
 *                      2 (64-bit key slots; fanout/keys_per_lane 2 or 4): as 1,
 *                      but planb_lookup and planb_lookup_index (on batches of
 *                      2^20 addresses or more; smaller ones run as 1) and the
 *                      persistent batch kernel (when it fits beside the batch
 *                      table) stage every internal level in LDS, ignoring
 *                      lds_levels: the bottom one as the top 32 bits of each
 *                      key, the levels above it whole, so that only the leaf is
 *                      read from device memory; a lookup whose address ties a
 *                      bottom key's top half reads that whole key (from the
 *                      first slot of the leaf it starts).
 *                      The many-FIB and IPv4 paths run this tuning as 1 with
 *                      lds_levels.  PLANB_ERANGE when those tops exceed a
 *                      workgroup's LDS.
 * A FIB starts with keys_per_lane = fanout/4 (or planb_params_t's), the
 * deepest lds_levels within 64 KiB, 2 lookups per group and the fastest
 * lds_search that applies: 2 with 1024 threads, else 1, else 0 (512 threads).
 */
typedef struct planb_tuning {
    uint32_t keys_per_lane;
    int32_t lds_levels;
    uint32_t lookups_per_group;
    uint32_t block_threads;
    uint32_t lds_search;
} planb_tuning_t;

/* Returns PLANB_EINVAL for an unsupported combination, PLANB_ERANGE when the
 * LDS levels exceed what a workgroup may allocate. */
int planb_set_tuning(planb_fib_t* fib, const planb_tuning_t* tuning);
int planb_get_tuning(const planb_fib_t* fib, planb_tuning_t* tuning);

/*
 * Pure layout arithmetic (Section 3, "Search on Linearized B+-Tree" closed
 * forms and "Parameter Tuning"), no allocation: for m keys, fanout b and
 * `slots` key slots per node, fills info->depth (smallest D with
 * (b-1) * b^(D-1) >= m), level_nodes and level_offset.  trimmed = 0 keeps every
 * internal node of a complete b-ary tree (the paper's layout, where level d
 * starts at node (b^d - 1)/(b - 1)); trimmed = 1 drops trailing internal nodes
 * that hold only sentinels.  Trailing all-sentinel leaves are never counted.
 * info->key_bytes is nodes * slots * 16.
 */
int planb_layout(uint64_t m, uint32_t fanout, uint32_t slots, int trimmed, planb_info_t* info);

/*
 * Uneven batches in one persistent launch (Section 3 "Batching": many
 * independent lookups in flight; here a grid of compute units x resident
 * workgroups stages the top levels in LDS once and then walks every batch).
 */
typedef struct planb_batch {
    const planb_addr_t* addrs; /* device, n records, 16-byte aligned */
    uint16_t* out;             /* device, n next hops, 2-byte aligned */
    uint64_t n;                /* may be 0 */
} planb_batch_t;

/* batches: device array of max_batches descriptors; n_batches: device pointer
 * to the number of valid descriptors (values above max_batches are clipped),
 * read by the kernel, so one launch shape serves any batch list.  The total
 * number of lookups per call must stay below 2^32.  Uses the FIB's current
 * tuning; its LDS levels plus 4 * (max_batches + block_threads + 1) bytes must
 * fit a workgroup's LDS (else PLANB_ERANGE). */
int planb_lookup_batches(const planb_fib_t* fib, const planb_batch_t* batches, const uint32_t* n_batches,
                         uint32_t max_batches, void* stream);

/*
 * The same persistent launch captured once into HIP graphs and replayed:
 * planb_graph_create captures (copy of a pinned host descriptor buffer to the
 * device) + (persistent batches kernel) for the FIB's current tuning, into a
 * ring of 4 graphs.  planb_graph_launch copies the host batch list into the
 * next ring slot's pinned buffer (waiting first, if that slot's previous
 * replay has not finished) and replays that slot's graph on `stream`; the
 * descriptors are read when the graph runs, the address and output buffers
 * must stay valid until it completes.  Later tuning changes do not affect an
 * existing graph.  planb_graph_free waits for outstanding replays.
 */
typedef struct planb_graph planb_graph_t;
planb_graph_t* planb_graph_create(const planb_fib_t* fib, uint32_t max_batches);
int planb_graph_launch(planb_graph_t* graph, const planb_batch_t* batches, uint32_t n_batches, void* stream);
void planb_graph_free(planb_graph_t* graph);

/*
 * Lookup autotuner: times every compiled-in tuning (keys per lane, lookups per
 * group, block size, the three deepest LDS depths that fit) on a device
 * sample of addresses with HIP events on `stream` (one warm-up plus `reps`
 * timed calls each, 0 -> 3), applies the fastest to the FIB and reports it.
 * The fanout is a build parameter; compare fanouts by building each.
 */
typedef struct planb_autotune_result {
    planb_tuning_t tuning;
    float ms_per_call;
    float glps;          /* sample lookups per second / 1e9 */
    uint32_t candidates; /* tunings timed */
} planb_autotune_result_t;

int planb_autotune(planb_fib_t* fib, const planb_addr_t* sample, size_t n, uint32_t reps, void* stream,
                   planb_autotune_result_t* result);

/*
 * Launch shapes by call size (uneven batches, the paper's Section 3
 * "Batching": a shape that suits 2^28 lookups is not the one for 64).
 * planb_set_size_tunings installs count entries with strictly ascending
 * min_lookups; planb_lookup and planb_lookup_index then run a call of n
 * lookups with the tuning of the last entry whose min_lookups <= n, and with
 * the FIB's own tuning (planb_set_tuning) below the first.  count = 0 clears
 * the table.  Each tuning is checked as by planb_set_tuning (PLANB_EINVAL,
 * PLANB_ERANGE; the table is unchanged on error).  Not synchronised with
 * lookups running on other host threads.  planb_get_size_tunings copies up
 * to cap entries (either array may be NULL) and returns the entry count.
 *
 * planb_autotune_sizes runs the autotuner (as planb_autotune, also trying
 * shallower LDS staging below 2^16 lookups) on the first sizes[k] addresses
 * of the device sample for each of count strictly ascending sizes (each in
 * 1..n), reports bucket k's winner in results[k], and installs them as size
 * tunings: bucket k serves calls from ceil(sqrt(sizes[k-1] * sizes[k]))
 * lookups up (bucket 0 from 1).  The FIB's own tuning is left as it was.
 */
int planb_set_size_tunings(planb_fib_t* fib, const uint64_t* min_lookups, const planb_tuning_t* tunings,
                           uint32_t count);
int planb_get_size_tunings(const planb_fib_t* fib, uint64_t* min_lookups, planb_tuning_t* tunings, uint32_t cap);
int planb_autotune_sizes(planb_fib_t* fib, const planb_addr_t* sample, size_t n, const uint64_t* sizes, uint32_t count,
                         uint32_t reps, void* stream, planb_autotune_result_t* results);

/*
 * Learned position model (an addition to the paper's method).  A
 * 16 -> 64 -> 64 -> 1 ReLU MLP reads the 16 address bytes (most significant
 * first) as byte/256 and predicts y ~ (interval index + 1/2) / m; W1, W2 and
 * w3 are bfloat16, biases float32, products run on MFMA with float32
 * accumulation.  Predicted position p = clamp(floor(y * m), 0, m - 1).  The
 * error table splits [0, m) into equal segments by p and stores, per segment,
 * the largest |p - i| over the first and last address of every interval and
 * two addresses drawn uniformly inside it (4m seeded points, evaluated by the
 * same inference kernel); training uses the same kind of points.
 * Trees with 64-bit key slots whose leaf tops fit a workgroup's LDS (the top
 * 32 bits of every leaf's first key, 4 bytes per leaf, built once with the
 * model, plus the error table): the window [p - w, p + w], w = 2 eps + 16,
 * becomes a range of leaves; a binary search over their tops finds the leaf,
 * verified on the tops (the range's first leaf starts at or below x's top
 * half, the leaf after it above), ties settled with whole keys; lane groups
 * then read that one leaf.  Other trees: with the window w = eps + eps/2 + 16
 * of interval positions, x's interval is found by descending the smallest
 * subtree that holds the leaves of lo and hi, and the result is accepted
 * unless the leaf reached counts no key <= x (x below the subtree) or counts
 * every key of the subtree's last leaf while another leaf follows (x may lie
 * beyond the subtree).  A lookup's error-table segment is estimated in float
 * arithmetic (within one of the exact one; a neighbouring segment's bound
 * only narrows or widens the window, which the check covers).  A lookup that
 * fails its check runs the tree descent, so results are always those of
 * planb_lookup.
 */
typedef struct planb_train_cfg {
    uint32_t epochs;   /* passes over the 4m sample points (0 -> about 30,000 steps in all, 8..400 passes) */
    uint32_t batch;    /* points per Adam step, a multiple of 16 (0 -> 4m/32, within 64..4096) */
    float lr;          /* peak Adam step size, cosine-decayed (0 -> 3e-3) */
    uint32_t segments; /* error-table segments (0 -> 4096); capped at m/64 */
    uint64_t seed;     /* initialisation and sample order */
} planb_train_cfg_t;

typedef struct planb_train_report {
    float final_loss;        /* mean squared error over the 4m points */
    uint32_t steps;          /* Adam steps taken */
    float seconds;           /* wall time of planb_train */
    uint32_t max_eps;        /* largest error bound over non-empty segments */
    float mean_eps;          /* mean error bound over non-empty segments */
    uint32_t empty_segments; /* segments no point predicts into (searched over the whole tree) */
} planb_train_report_t;

/* Trains the FIB's model from scratch with the hand-written kernels (forward,
 * backward and Adam; per-workgroup gradient partials reduced in a fixed
 * order, so a seed gives the same model every run), then builds the error
 * table.  Synchronises `stream`.  report may be NULL.  PLANB_ERANGE for a FIB
 * of 2^32 or more intervals (here and in planb_model_set_params): the learned
 * kernels keep positions in 32 bits. */
int planb_train(planb_fib_t* fib, const planb_train_cfg_t* cfg, void* stream, planb_train_report_t* report);

/* Exact lookup through the model (see above).  From 2^21 lookups (2^18 when
 * the tree does not take the leaf-tops kernel) the lookups whose window check
 * fails are appended to a fallback queue in scratch device memory (a counter
 * and one 4-byte entry per lookup: 256 + 4n bytes, allocated with
 * hipMallocAsync on `stream` and freed with hipFreeAsync behind the work, so
 * the host never waits); a second kernel then runs the tree descent for the
 * queued lookups.  Smaller calls run one kernel, in which such lookups
 * descend the tree in place, and allocate nothing.  fallback_count (device
 * uint32, may be NULL) is incremented by the number of lookups that fell
 * back -- the caller zeroes it.
 *   addrs  device, n records, 16-byte aligned;  out: device, n uint16
 *   n      0 is a no-op; must be < 2^32
 * Returns PLANB_OK, PLANB_EINVAL (no trained model, NULL or misaligned
 * pointer), PLANB_ERANGE, PLANB_ENOMEM (the queue could not be allocated),
 * PLANB_EDEVICE. */
int planb_lookup_learned(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint16_t* out,
                         uint32_t* fallback_count, void* stream);

/* planb_lookup_learned for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors, but the fallback queue is a
 * fixed device array of the library (16 MiB + 256 bytes on each GPU it runs
 * on, held until the process ends) instead of an allocation, so the call
 * makes no hipMalloc/hipMallocAsync/hipFree and no allocating library call.
 *   n  at most 4,194,304 (2^22) lookups per call; more gives PLANB_ERANGE.
 * Every call on one GPU shares that array, which keeps the last call's
 * contents (a kernel clears its counter at the start of each call): calls
 * that overlap on one GPU -- on different streams, or from different host
 * threads without ordering -- race and may return wrong next hops.  Order
 * them on one stream. */
int planb_lookup_learned_noalloc(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint16_t* out,
                                 uint32_t* fallback_count, void* stream);

/* Model access (tests, checkpoints).  The flat parameter vector holds W1
 * (64 x 16, row-major), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1):
 * planb_model_num_params() floats.  set_params creates the model if needed,
 * resets the Adam state and leaves every segment "empty" (whole-tree searches)
 * until planb_model_build_eps or planb_model_set_eps. */
int planb_model_num_params(void);
int planb_model_set_params(planb_fib_t* fib, const float* params, uint32_t segments);
int planb_model_get_params(const planb_fib_t* fib, float* params);
/* y (device, n floats): raw model output for each address. */
int planb_model_predict(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, float* y, void* stream);
/* grad (device, num_params floats): gradient of mean((y - t)^2) over the n
 * device samples/targets at the current weights (no update). */
int planb_model_grad(planb_fib_t* fib, const planb_addr_t* samples, const float* targets, size_t n, float* grad,
                     void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with a
 * device gradient on the float32 master weights; refreshes the bf16 copy. */
int planb_model_adam(planb_fib_t* fib, const float* grad, float lr, void* stream);
int planb_model_build_eps(planb_fib_t* fib, void* stream);
/* Error table to / from host memory; 0xFFFFFFFF marks an empty segment. */
int planb_model_get_eps(const planb_fib_t* fib, uint32_t* eps, uint32_t cap);
int planb_model_set_eps(planb_fib_t* fib, const uint32_t* eps, uint32_t n);

/*
 * Several FIBs in one launch.  A table set is a device array of tree
 * descriptors (slot -> FIB); every FIB in a set must share fanout and key
 * width.  planb_lookup_multi walks a device list of bursts, each naming its
 * slot, in one persistent launch (tiles as in planb_lookup_batches; all tree
 * levels are read through the caches).  Bursts naming an empty or
 * out-of-range slot are skipped (their outputs are not written).
 */
typedef struct planb_burst {
    uint32_t table;            /* slot in the table set */
    uint32_t n;                /* addresses in the burst */
    const planb_addr_t* addrs; /* device, 16-byte aligned */
    uint16_t* out;             /* device, 2-byte aligned */
} planb_burst_t;

typedef struct planb_tableset planb_tableset_t;
planb_tableset_t* planb_tableset_create(uint32_t max_tables);
/* Points slot at fib (NULL empties it).  Launches of the set already
 * enqueued read the descriptors when they run, so the call first waits (on
 * the host) for those launches to finish, then writes the slot.  The caller
 * keeps fib alive while the slot names it. */
int planb_tableset_set(planb_tableset_t* ts, uint32_t slot, const planb_fib_t* fib);
/* Launch shape of the multi-FIB kernel (keys per lane, lookups per group, block size). */
int planb_tableset_set_tuning(planb_tableset_t* ts, uint32_t keys_per_lane, uint32_t lookups_per_group,
                              uint32_t block_threads);
/* 4 * (max_bursts + block_threads + 1) bytes of LDS must fit a workgroup. */
int planb_lookup_multi(const planb_tableset_t* ts, const planb_burst_t* bursts, const uint32_t* n_bursts,
                       uint32_t max_bursts, void* stream);
/* The learned lookup (planb_lookup_learned) for each burst whose FIB has a
 * trained model (the model as it was when the FIB was set into the slot: set
 * it again after training), the tree descent for the others; results are
 * those of planb_lookup_multi.  fallback_count (device u32, may be NULL) is
 * increased by the number of learned lookups that fell back to the tree.
 * Descriptors as for planb_lookup_multi; LDS: 4 * (max_bursts + 257)
 * bytes must fit a workgroup. */
int planb_lookup_multi_learned(const planb_tableset_t* ts, const planb_burst_t* bursts, const uint32_t* n_bursts,
                               uint32_t max_bursts, uint32_t* fallback_count, void* stream);
void planb_tableset_free(planb_tableset_t* ts);

/*
 * Serving runtime (Section 3 "Batching" and "Dynamic FIB Update", Section 4's
 * RX-LPM-TX pipeline, for a GPU).  Tables are registered by id with their
 * rules and built on the device when a burst first needs them; while the
 * device memory budget would be exceeded, the least recently used tables with
 * no launch in flight are evicted (rebuilt on a later use).  Bursts are
 * queued by planb_server_submit; planb_server_poll finishes launches whose
 * completion event has fired (copying results to the callers' host buffers)
 * and packs queued bursts of any tables into every free launch slot, one
 * stream per slot, so arrivals join the next launch while others run
 * (continuous batching).  Each launch carries its own copy of the tree and
 * model descriptors of the tables it serves, so planb_server_set_table on a
 * live id (which swaps in the rebuilt FIB) and evictions never change what a
 * launch already enqueued reads; a replaced FIB is freed after the launches
 * that read it.  A burst whose table cannot be made resident (its rules fail
 * to build, or it alone exceeds the budget) completes at once with that
 * status and its output untouched.
 * Single-threaded: call a server's functions from one thread.
 */
typedef struct planb_server planb_server_t;

typedef struct planb_server_cfg {
    uint32_t max_tables;    /* table ids 0 .. max_tables-1 (0 -> 16) */
    uint32_t streams;       /* launch slots / streams in flight at once, 1..8 (0 -> 2) */
    uint32_t max_bursts;    /* bursts per launch (0 -> 1024) */
    uint32_t max_lookups;   /* addresses per launch (0 -> 2^20) */
    uint32_t fanout;        /* fanout of every table (0 -> 16) */
    uint32_t key_bits;      /* 32, 64 or 128 for every table (0 -> 128) */
    uint64_t memory_budget; /* device bytes for resident trees (0 = unlimited) */
    uint32_t learned;       /* 1: train a learned model (a short run: 8 passes) for every table when it is admitted and
                               serve bursts with planb_lookup_multi_learned (0: planb_lookup_multi) */
    uint32_t flags;         /* PLANB_SERVER_* (0: bursts staged through pinned copies) */
} planb_server_cfg_t;

/* Zero-copy serving: the lookup kernels read each burst's addresses from, and
 * write its next hops to, the caller's host memory directly over PCIe; there
 * are no staging copies on the host nor DMA copies per launch.  Every burst's
 * addrs and out must then lie in pinned host memory registered with
 * planb_server_register_io (planb_server_submit returns PLANB_EINVAL
 * otherwise).  Completion (poll) means the next hops are in out. */
#define PLANB_SERVER_ZERO_COPY 1u

typedef struct planb_completion {
    int64_t tag;      /* the submitter's tag */
    uint32_t table;
    uint32_t n;
    double submit_us; /* planb_server_now_us() at submit */
    double done_us;   /* ... when poll saw the launch complete */
    int32_t status;   /* PLANB_OK, or the error that kept the burst's table from being served */
    int32_t pad;
} planb_completion_t;

typedef struct planb_server_stats {
    uint64_t launches, bursts, lookups, admissions, evictions, resident_bytes;
    uint32_t resident_tables, queued;
} planb_server_stats_t;

planb_server_t* planb_server_create(const planb_server_cfg_t* cfg);
void planb_server_free(planb_server_t* server); /* waits for launches in flight */
/* Registers or replaces table id (the rules are validated and copied). */
int planb_server_set_table(planb_server_t* server, uint32_t id, const planb_addr_t* prefixes,
                           const uint8_t* lengths, const uint16_t* next_hops, size_t n);
/* Queues a burst: addrs (host, n records) must stay valid and unchanged, and
 * out (host, n uint16) is written, until poll returns the burst's completion
 * (the addresses are copied to pinned staging when the burst joins a launch,
 * so submitting costs no copy; with PLANB_SERVER_ZERO_COPY the kernels read
 * and write the caller's registered buffers themselves). */
int planb_server_submit(planb_server_t* server, uint32_t table, const planb_addr_t* addrs, uint32_t n,
                        uint16_t* out, int64_t tag);
/* Registers [base, base + bytes) as I/O memory for zero-copy bursts.  It must
 * be pinned host memory the device can address at the same addresses
 * (hipHostMalloc, or a pinned torch tensor), within one allocation;
 * PLANB_EINVAL otherwise.  At most 64 ranges; the memory must stay allocated
 * while the server may use it. */
int planb_server_register_io(planb_server_t* server, const void* base, size_t bytes);
/* Progresses the server and returns up to cap completions (count >= 0 or a
 * status).  block != 0 waits until at least one completion is available or
 * nothing is queued or in flight. */
int planb_server_poll(planb_server_t* server, planb_completion_t* out, uint32_t cap, int block);
int planb_server_stats(const planb_server_t* server, planb_server_stats_t* stats);
double planb_server_now_us(void);
/* Makes table id resident now (evicting idle tables if the budget needs it). */
int planb_server_admit(planb_server_t* server, uint32_t id);
/* Open-loop load generator beside the server: burst k arrives at
 * start + arrival_us[k] (start = now + 1 ms), is submitted then, and its
 * latency_us[k] runs from that arrival to the poll that sees it complete.
 * addrs / out (host) hold all bursts back to back, burst k at
 * [offsets[k], offsets[k+1]) (n_bursts + 1 offsets); arrivals and offsets are
 * non-decreasing.  *wall_s (may be NULL) receives the elapsed seconds. */
int planb_server_replay(planb_server_t* server, uint32_t n_bursts, const double* arrival_us, const uint32_t* table,
                        const uint64_t* offsets, const planb_addr_t* addrs, uint16_t* out, double* latency_us,
                        double* wall_s);

/*
 * Host-only halves of planb_build, usable without a GPU (tools, tests).
 *
 * planb_build_intervals -- range conversion and interval partitioning
 * (Section 3, "From 2D Prefixes to 1D Intervals"; Algorithm 2's sweep): the
 * same validation and steps as planb_build up to the elementary intervals.
 * Writes min(m, cap) starts / next hops to host memory (either may be NULL)
 * and returns m, or a negative planb_status.  flags: PLANB_FLAG_*.
 */
long long planb_build_intervals(const planb_addr_t* prefixes, const uint8_t* lengths,
                                const uint16_t* next_hops, size_t n, uint32_t flags,
                                planb_addr_t* starts, uint16_t* next_hops_out, size_t cap);

/*
 * planb_build_keys -- the linearized B+-tree key array (Section 3, "Linearized
 * B+-Tree", "Maintaining Structural Integrity", Algorithm 2's leaf fill and
 * separator pass) for m strictly increasing interval starts (starts[0] == 0),
 * laid out as planb_build lays out a FIB with 128-bit keys: internal nodes of
 * `fanout` 16-byte slots (fanout-1 keys + one sentinel 2^128-1 slot), levels
 * top-down, trailing all-sentinel nodes dropped, then the leaves (see
 * planb_info_t; here every slot a built FIB fills with next hops holds the
 * sentinel).  keys: host, cap_keys records; info (may be NULL) receives the
 * shape.  Returns the number of slots (may exceed cap_keys, then nothing is
 * written) or a negative status.
 */
long long planb_build_keys(const planb_addr_t* starts, size_t m, uint32_t fanout,
                           planb_addr_t* keys, size_t cap_keys, planb_info_t* info);

/*
 * planb_build_image -- the exact device slot array planb_build uploads for m
 * strictly increasing interval starts (starts[0] == 0) and their next hops:
 * the key array above in key_bits-wide slots (64: the high word of each key,
 * 32: its top 32 bits; 0 picks the narrowest exact width, as planb_build
 * does) with every leaf carrying its next hops (see planb_info_t).  With
 * 64-bit slots a leaf is a run of 32-byte blocks of three keys and their
 * three uint16 next hops, with 32-bit slots of five keys and five hops; with
 * 128-bit slots the keys come first, then the next hops.  Slots past the last
 * interval hold the all-ones sentinel and next hop 0xFFFF.
 * image: host, cap_bytes bytes; info (may be NULL) receives the shape.
 * Returns the image size in bytes (may exceed cap_bytes, then nothing is
 * written) or a negative status.
 */
long long planb_build_image(const planb_addr_t* starts, const uint16_t* next_hops, size_t m, uint32_t fanout,
                            uint32_t key_bits, void* image, size_t cap_bytes, planb_info_t* info);

/*
 * planb_cpu_lookup -- host-core baseline: the linearized B+-tree lookup of
 * Section 3 (Algorithm 1, with the paper's batching and branch-free node
 * search) run on the CPU over the image planb_build_image returns (info: the
 * shape it reported).  addrs/out: host arrays of n records.  threads <= 0
 * uses every hardware thread.  For measurements beside the GPU kernel only;
 * no GPU entry point calls it.  Returns PLANB_OK or PLANB_EINVAL.
 */
int planb_cpu_lookup(const void* image, const planb_info_t* info, const planb_addr_t* addrs, size_t n,
                     uint16_t* out, int threads);

/*
 * planb_cpu_tree_* -- host-core baseline in the paper's own CPU design
 * (Section 3: "Parameter Tuning" b = 9, so 8 keys per 64-byte node;
 * "Separation of Keys and Values"; Algorithm 1 and Listing 1's count of keys
 * <= x per node by one vector compare and a popcount, "Vectorization and SIMD
 * Acceleration"; "Batching"; "Branch-Free Traversal and Loop Unrolling").
 * planb_cpu_tree_build lays out a fanout-9 linearized B+-tree over m sorted
 * interval starts (host; starts[0] must be 0, strictly increasing) and keeps
 * a copy of their next hops; key_bits is 64 (the paper's width: only exact,
 * and only accepted, when every start's low word is zero) or 128 (a node's 8
 * high words, then its 8 low words).  NULL on bad input or allocation failure.
 * planb_cpu_tree_lookup searches n host addresses into n host next hops with
 * `threads` threads (<= 0: every hardware thread), AVX-512 compares when the
 * host has them, else AVX2 (planb_cpu_tree_isa says which: "avx512" or
 * "avx2"); PLANB_OK or PLANB_EINVAL.  Host only: for measurements beside the
 * GPU kernels; no GPU entry point calls it.
 */
typedef struct planb_cpu_tree planb_cpu_tree_t;
planb_cpu_tree_t* planb_cpu_tree_build(const planb_addr_t* starts, const uint16_t* next_hops, size_t m,
                                       uint32_t key_bits);
int planb_cpu_tree_lookup(const planb_cpu_tree_t* tree, const planb_addr_t* addrs, size_t n, uint16_t* out,
                          int threads);
const char* planb_cpu_tree_isa(const planb_cpu_tree_t* tree);
int planb_cpu_tree_depth(const planb_cpu_tree_t* tree);
void planb_cpu_tree_free(planb_cpu_tree_t* tree);

#ifdef __cplusplus
}
#endif
#endif /* PLANB_H */
