/*
 * polar_scl.h -- C ABI of the MI355X (gfx950) flexible CRC-aided SCL polar
 * decoder.
 *
 * The method is that of Leonardon, Cassagne, Leroux, Jego, Hamelin and
 * Savaria, "Fast and Flexible Software Polar List Decoders"
 * (arXiv:1710.08314): successive-cancellation list decoding (Algorithm 1,
 * Sec. II-B2) with the Rate-0 / Rate-1 / repetition / single-parity-check
 * dedicated nodes (Sec. II-B3), CRC-aided selection (Sec. II-B4, Sec. IV-B),
 * fully / partially adaptive list sizes (Sec. II-B5) and float32, 16-bit and
 * 8-bit saturated arithmetic (Sec. III-B3).  Every code and decoder parameter
 * (Sec. III-A, III-B) is a runtime value of a plan; nothing is recompiled.
 *
 * Conventions shared by every entry point
 *   - Return value: 0 on success or a negative POLAR_E* code; no exception
 *     crosses the boundary.  polar_strerror() names a code.
 *   - Pointers named d_* are device (HBM) pointers owned by the caller; all
 *     other pointers are host pointers, read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls that take a stream only enqueue work on it and return without
 *     waiting; the caller synchronises before reading outputs.
 *   - Bit vectors are packed little-endian in 32-bit words: bit j of a vector
 *     is bit (j % 32) of word j / 32.
 *   - A plan is immutable after creation and may be shared by several
 *     streams and host threads; it owns device tables until destroyed.
 */
#ifndef POLAR_SCL_H
#define POLAR_SCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define POLAR_OK 0
#define POLAR_EINVAL (-1)    /* invalid argument or inconsistent descriptor      */
#define POLAR_EUNSUP (-2)    /* valid but outside what the GPU decoder supports  */
#define POLAR_ENOMEM (-3)    /* device or host allocation failed                 */
#define POLAR_EHIP (-4)      /* a HIP runtime call failed                        */
#define POLAR_ENOTSYS (-5)   /* frozen set unusable for systematic encoding      */
#define POLAR_EAGAIN (-6)    /* serving: no free slot or budget right now; poll  */
#define POLAR_ESCRATCH (-7)  /* polar_scl_decode_batch_noalloc: the batch needs
                              * more than its fixed device area                  */

/* ------------------------------------------------------------ enumerations */
/* LLR / path-metric arithmetic (Sec. III-B3).  Integer modes saturate to
 * [-127, 127] and [-32767, 32767] after every operation. */
typedef enum { POLAR_F32 = 0, POLAR_I16 = 1, POLAR_I8 = 2 } polar_quant;

/* Decoding algorithm (Sec. II-B, Table I).  SC is the L = 1 decoder; CA_SCL a
 * fixed list size L; PA_SCL the stages 1 then L_max; FA_SCL the stages
 * 1, 2, 4, ... up to L_max, each restarted from the channel LLRs when no
 * candidate of the previous stage passes the CRC. */
typedef enum { POLAR_SC = 0, POLAR_CA_SCL = 1, POLAR_PA_SCL = 2, POLAR_FA_SCL = 3 } polar_algo;

/* Dedicated nodes that prune the decoding tree (Sec. II-B3, Sec. III-B2). */
enum { POLAR_NODE_R0 = 1, POLAR_NODE_R1 = 2, POLAR_NODE_REP = 4, POLAR_NODE_SPC = 8 };
#define POLAR_NODE_ALL 15u

/* ------------------------------------------------------------------- plans */
/* Descriptor of a code and its decoder (Sec. III-A genericity, Sec. III-B
 * flexibility).  All fields are runtime parameters. */
typedef struct {
  uint32_t N;           /* mother code length, a power of two, 2 <= N <= 2048        */
  uint32_t K;           /* |A|: information positions INCLUDING the crc_len CRC bits */
  const uint32_t *frozen;   /* host, ceil(N/32) words, bit i = 1: u_i frozen; or NULL:
                             * the |A| most reliable positions by the Bhattacharyya
                             * recursion at design_ebn0_db                            */
  float design_ebn0_db; /* construction point when frozen == NULL                     */
  uint32_t n_shorten;   /* S: codeword positions [N-S, N) are known zeros, not sent;
                         * u-indices [N-S, N) must be (or are made) frozen           */
  uint32_t crc_len;     /* c, 0..32 (0: no CRC; then PA/FA are rejected)             */
  uint64_t crc_poly;    /* generator g(x): the c low coefficients (an x^c term, if
                         * present, is ignored); MSB-first, init 0, no final xor    */
  uint32_t algo;        /* polar_algo                                                */
  uint32_t L;           /* list size for CA_SCL (power of two, 1..32)                */
  uint32_t L_max;       /* last stage for PA/FA (power of two, 1..32)                */
  uint32_t quant;       /* polar_quant of the LLRs handed to the decoder             */
  uint32_t node_enable; /* OR of POLAR_NODE_*                                        */
  uint32_t rep_max;     /* largest REP node (0 = unlimited; 8 gives REP8-)           */
  uint32_t spc_max;     /* largest SPC node (0 = unlimited; 4 gives SPC4)            */
  uint32_t r1_max;      /* largest Rate-1 node (0 = unlimited)                       */
  uint32_t r0_max;      /* largest Rate-0 node (0 = unlimited)                       */
  uint32_t n_puncture;  /* P: codeword positions [0, P) are not sent and decode as
                         * LLR 0; u-indices [0, P) must be (or are made) frozen; the
                         * sent LLRs are positions [P, N - S)                         */
} polar_plan_desc;

typedef struct polar_plan_s *polar_plan;

/* Build a plan: frozen set (given or constructed), systematic-encoding check,
 * the pre-order program of the pruned decoding tree, CRC tables, and their
 * upload to device memory (synchronous, on the current device).
 * Errors: POLAR_EINVAL (bad sizes, K > N - S, frozen mask with |A| != K, a
 * frozen mask that leaves a shortened u-index unfrozen), POLAR_EUNSUP (N >
 * 2048, L or L_max > 32 or not a power of two, crc_len > 32, float32 at a
 * list size whose decoder state exceeds the LDS of one CU), POLAR_ENOTSYS
 * (the systematic encoder of Sec. II-A would not give x_A = b for this
 * frozen set), POLAR_ENOMEM, POLAR_EHIP.  *out is written only on success. */
int polar_scl_plan(const polar_plan_desc *desc, polar_plan *out);

/* Release a plan and its device tables.  The caller guarantees that no work
 * using the plan is still pending on any stream.  NULL is accepted. */
int polar_plan_destroy(polar_plan p);

/* Sizes a caller needs to lay out buffers for a plan. */
typedef struct {
  uint32_t N, K, crc_len, n_tx;  /* n_tx = N - S transmitted positions                */
  uint32_t k_data;               /* K - crc_len decoded information bits per frame    */
  uint32_t info_words;           /* ceil(k_data / 32): d_info words per frame         */
  uint32_t code_words;           /* ceil(N / 32): polar_encode words per frame        */
  uint32_t llr_bytes;            /* n_tx * element size of the plan's quant           */
  uint32_t max_list;             /* largest list size the plan's schedule reaches     */
  uint32_t n_ops;                /* length of the node program                        */
  uint32_t n_r0, n_r1, n_rep, n_spc, n_leaf_frozen, n_leaf_info; /* pruned-tree nodes */
  uint32_t lds_bytes;            /* decoder LDS footprint per frame at max_list       */
} polar_plan_info;

int polar_plan_get_info(polar_plan p, polar_plan_info *out);

/* Copy the plan's frozen mask (ceil(N/32) host words, bit = 1: frozen). */
int polar_plan_get_frozen(polar_plan p, uint32_t *frozen_words);

/* Host-only dry run of polar_scl_plan: validates the descriptor and fills
 * *info and (if non-NULL) the frozen mask exactly as the plan would, without
 * touching any device.  Same error codes as polar_scl_plan except POLAR_EHIP
 * and POLAR_ENOMEM. */
int polar_plan_query(const polar_plan_desc *desc, polar_plan_info *info, uint32_t *frozen_words);

/* ------------------------------------------------------------------ decode */
/* One frame of a batch (device array).  llr_off: byte offset of its n_tx
 * LLRs in d_llr (aligned to the element size); out_off: word offset of its
 * info_words output words in d_info; plan_idx: index into `plans`. */
typedef struct {
  uint64_t llr_off;
  uint32_t out_off;
  uint32_t plan_idx;
} polar_frame;

/* Per-frame result (device array, one per frame). */
typedef struct {
  uint8_t crc_ok;   /* 1: the output passed the CRC (always 1 without a CRC)     */
  uint8_t L_used;   /* list size of the stage whose output was taken              */
  uint8_t n_paths;  /* paths alive at the end of that stage                       */
  uint8_t flags;    /* bit 0 (POLAR_STATUS_NEAR_TIE), float32 plans only: some
                     * decision of the decode -- a selection of the L best
                     * candidates (Sec. II-B2), or the final CRC choice in
                     * metric order (Sec. II-B4) -- separated the kept path from
                     * a rejected or passed-over one by a metric gap of at most
                     * 1e-4 max(1, |metric|), in any stage run (Sec. II-B5);
                     * another float rounding could then decide otherwise.
                     * Always 0 in the integer modes.  Other bits 0.         */
  uint32_t pm;      /* path metric of the output: float32 bits, or int32 value    */
} polar_status;
#define POLAR_STATUS_NEAR_TIE 1u

/* opts->flags: record HIP events on `stream` around every kernel launch of
 * the call (see polar_last_tier_ms). */
#define POLAR_OPT_TIER_TIMING 1u
/* opts->flags: for a batch of fixed-list plans (class schedule, below), time
 * the candidate schedules on this very batch the first time its plan list is
 * seen, keep the fastest in the library's schedule cache (keyed by the plan
 * list) and use it from then on.  The call then blocks until the candidates
 * have run; its outputs are those of the chosen schedule (every candidate
 * computes the same outputs).  Not usable under graph capture. */
#define POLAR_OPT_AUTOTUNE 2u

/* Optional knobs; NULL selects defaults. */
typedef struct {
  uint32_t schedule;   /* 0 = automatic: a batch of fixed-list plans (CA-SCL, SC)
                        * with several plans uses the class schedule -- frames
                        * split by list size and code length, one persistent
                        * kernel per class sized for that class; a batch of
                        * fewer than 32 frames with an adaptive plan runs the
                        * plain form; otherwise the tiered schedule -- an L = 1
                        * tier, then the list stages, each frame's next list
                        * size kept in a per-frame state word on the device.
                        * 1 = plain (one generic launch in which each workgroup
                        * runs whole frames, every stage in place)                */
  uint32_t flags;      /* OR of POLAR_OPT_*                                         */
  uint64_t *d_times;   /* nullable device array, 2 per frame: the device realtime
                        * counter (polar_device_clock_khz) when the frame's decode
                        * starts and when its outputs are written                 */
  uint32_t reserved[4];
} polar_decode_opts;

/* Decode a batch (the hot path, Algorithm 1 and Sec. II-B3..B5).
 *   plans[n_plans]   host array of plans used by the frames: all of one quant,
 *                    except that a batch of two or more fixed-list plans (CA-SCL,
 *                    SC) in the automatic schedule may mix them (each frame's
 *                    LLRs then in its own plan's type, at its descriptor's
 *                    llr_off)
 *   d_frames         device array of n_frames descriptors, or NULL: then every
 *                    frame uses plans[0], frame f reads d_llr + f * llr_bytes
 *                    and writes d_info + f * info_words
 *   d_llr            channel LLRs, natural codeword order, in the plans' quant
 *                    type (LLR > 0 favours bit 0); shortened positions are not
 *                    included
 *   d_info           decoded information bits (k_data per frame, packed)
 *   d_status         n_frames polar_status
 *   d_pm_lists       nullable; per frame max_list uint32 (float32 bits or int32):
 *                    the final path metrics in ascending order, unused entries
 *                    0xFFFFFFFF
 *   scratch          the library keeps a per-device work area (per-frame state
 *                    words, frame lists, counters, spill regions) that grows on
 *                    demand: concurrent calls on different streams of one
 *                    device must be serialised by the caller.
 * Errors: POLAR_EINVAL (NULL buffers, mixed quants outside the case above; a
 * plan index out of range is not checked on device: the caller guarantees
 * it), POLAR_EHIP. */
int polar_scl_decode_batch(const polar_plan *plans, uint32_t n_plans,
                           const polar_frame *d_frames, uint32_t n_frames,
                           const void *d_llr, uint32_t *d_info, polar_status *d_status,
                           uint32_t *d_pm_lists, const polar_decode_opts *opts, void *stream);

/* Allocation-free decode, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, outputs and kernels as polar_scl_decode_batch
 * (opts->flags may not contain POLAR_OPT_TIER_TIMING or POLAR_OPT_AUTOTUNE:
 * both create events; POLAR_EINVAL), but the call allocates nothing: its
 * plan table, work area and spill regions live in a fixed device area of
 * 96 MiB that the library holds once per GPU until the process ends (its
 * address is looked up at the first polar_scl_plan on each device).
 * Persistent grids are cut so that their spill regions fit the area, so a
 * large batch may run on fewer workgroups than polar_scl_decode_batch uses.
 * Limits: n_frames <= 2^21 and n_plans <= 16384, and the batch's largest
 * spill region must fit; otherwise POLAR_ESCRATCH and nothing is enqueued.
 * Every call on a GPU uses that GPU's one area and leaves its contents
 * behind (each call clears what must start at zero with its own kernels):
 * calls that overlap on one GPU -- on different streams, or from several
 * host threads -- race and must be serialised by the caller. */
int polar_scl_decode_batch_noalloc(const polar_plan *plans, uint32_t n_plans,
                                   const polar_frame *d_frames, uint32_t n_frames,
                                   const void *d_llr, uint32_t *d_info, polar_status *d_status,
                                   uint32_t *d_pm_lists, const polar_decode_opts *opts,
                                   void *stream);

/* ---------------------------------------------------- encoder and channel */
/* Systematic encoding with CRC attachment (Sec. II-A, Sec. II-B4): per frame,
 * b = data || CRC(data), u_A = b, u' = u F, u'_{A^c} = 0, x = u' F.
 *   d_data: n_frames * info_words words (k_data bits per frame, packed)
 *   d_code: n_frames * code_words words (N codeword bits; the transmitted
 *           part is bits [0, n_tx), the shortened tail is always zero). */
int polar_encode(polar_plan p, const uint32_t *d_data, uint32_t *d_code, uint32_t n_frames,
                 void *stream);

/* Workload generator of the Monte-Carlo chain (Sec. II-C), not part of the
 * decoder: i.i.d. data bits (d_data, info_words per frame) for frames
 * [frame0, frame0 + n_frames) of stream `seed`, counter-based (Philox4x32-10),
 * so any range can be regenerated independently. */
int polar_gen_data(polar_plan p, uint64_t seed, uint64_t frame0, uint32_t n_frames,
                   uint32_t *d_data, void *stream);

/* BPSK (0 -> +1) over AWGN at Eb/N0 (rate R = k_data / n_tx, sigma^2 =
 * 1 / (2 R Eb/N0)), LLR = 2 y / sigma^2, quantised to the plan's type as
 * clamp(rint(LLR * 2^frac_bits), -Q, Q) (float32: rounded to nearest).
 * Writes n_tx LLRs per frame contiguously into d_llr.  Noise is Philox4x32-10
 * + Box-Muller, counter-based on (seed, frame). */
int polar_channel(polar_plan p, const uint32_t *d_code, uint32_t n_frames, float ebn0_db,
                  int32_t frac_bits, uint64_t seed, uint64_t frame0, void *d_llr, void *stream);

/* The LLR quantiser of the fixed-point decoders (Sec. III-B3): n float32
 * LLRs (device) to the type of `quant` (polar_quant) in d_out (device, n
 * elements): q = clamp(rint(llr * 2^frac_bits), -Q, Q) with rounding half
 * to even, Q = 127 (int8, the paper's 6 integer + 2 fractional bits at
 * frac_bits = 2) or 32767 (int16); infinities saturate, NaN gives +Q;
 * POLAR_F32 copies.  Async on `stream`.  POLAR_EINVAL for a bad quant or
 * frac_bits outside 0..14. */
int polar_quantize(const float *d_llr, uint32_t n, int32_t quant, int32_t frac_bits, void *d_out,
                   void *stream);

/* Algorithmic work of one decoding stage of plan p at list size L, counted
 * from the node program and the deterministic growth of the active list
 * (a <- min(L, a * candidates) at every forking node): f and g LLR updates
 * (m/2 per path per node), h partial-sum updates (m/2 per path), node-level
 * penalty terms (m per path per dedicated node or leaf), candidate sorting
 * (C ceil(log2 C) comparisons for C candidates) and the final CRC checks
 * (|A| bits per surviving path).  *ops receives the element-operation count
 * (host only; no device work).  POLAR_EINVAL for L not a power of two or
 * above 32. */
int polar_plan_stage_work(polar_plan p, uint32_t L, uint64_t *ops);

/* Kernel durations (ms) of the last polar_scl_decode_batch call made with
 * POLAR_OPT_TIER_TIMING on this host thread: ms[0] the L = 1 tier, ms[1] list
 * tier A (L <= 4), ms[2] list tier B, ms[3] the plain kernel, ms[4] the
 * kernels of the class schedule together; 0 for what did not run.  Waits for
 * the recorded events.  POLAR_EINVAL if no timed call was made. */
int polar_last_tier_ms(float ms[5]);

/* Text description of the class schedule the library would use for this
 * plan list (classes, kernel variant, LDS bytes and workgroups of each, and
 * whether it came from POLAR_OPT_AUTOTUNE), NUL-terminated, truncated to
 * `len` bytes.  POLAR_EINVAL for an empty or NULL list or a list that does
 * not use the class schedule. */
int polar_schedule_describe(const polar_plan *plans, uint32_t n_plans, char *buf, uint32_t len);

/* ------------------------------------------------------------ HIP graphs */
/* A decode of fixed buffers captured once into a HIP graph and replayed:
 * polar_graph_create takes the arguments of polar_scl_decode_batch (same
 * meaning; opts->flags may not contain POLAR_OPT_TIER_TIMING or
 * POLAR_OPT_AUTOTUNE, a schedule cached by an earlier autotuned call is
 * used) and records the launches of one decode, with a work area of its own,
 * into an executable graph; polar_graph_launch replays it on `stream`,
 * decoding whatever the buffers hold at that time.  Buffers and plans must
 * outlive the graph.  Replays of one graph must not overlap. */
typedef struct polar_graph_s *polar_graph;
int polar_graph_create(const polar_plan *plans, uint32_t n_plans, const polar_frame *d_frames,
                       uint32_t n_frames, const void *d_llr, uint32_t *d_info,
                       polar_status *d_status, uint32_t *d_pm_lists,
                       const polar_decode_opts *opts, polar_graph *out);
int polar_graph_launch(polar_graph g, void *stream);
int polar_graph_destroy(polar_graph g);

/* -------------------------------------------------------------- serving */
/* Continuous batching of decode requests on one device.  A server owns
 * `n_slots` HIP streams, each with a work area for up to `max_batch` frames
 * and a fixed spill area, all allocated by polar_server_create.  A submitted
 * batch (a range of a caller's frame descriptors whose LLRs are already in
 * device memory) is admitted when a slot is free and the admission budget
 * holds it; it is then enqueued at once on the slot's stream, so batches
 * admitted while others run overlap on the device.  All decoding, including
 * the adaptive list escalation (Sec. II-B5), happens on the device without
 * host round trips; the host only admits and polls.
 *
 * Admission budget: frames in flight stay within `max_inflight`, and, with
 * budget_bytes > 0, the device bytes of the frames in flight stay within
 * budget_bytes, a frame being charged polar_plan_frame_bytes of its plan
 * (its LLRs, outputs, work-area words and the decoder state of its largest
 * list stage). */
typedef struct {
  uint32_t n_slots;       /* concurrent batches (HIP streams), 1..64             */
  uint32_t max_batch;     /* frames per batch                                    */
  uint32_t max_inflight;  /* frames admitted, not yet complete                   */
  uint32_t reserved;      /* 0                                                   */
  uint64_t budget_bytes;  /* 0: no byte budget; else the bytes admitted, not yet
                           * complete, stay within it                            */
  uint64_t slot_spill_bytes; /* spill area per slot (0: 64 MiB); persistent grids
                              * of a batch are cut to fit it, and a batch whose
                              * largest spill region does not fit is refused
                              * with POLAR_EUNSUP                                 */
} polar_server_config;

typedef struct polar_server_s *polar_server;

int polar_server_create(const polar_server_config *cfg, polar_server *out);

/* Device bytes one in-flight frame of plan p is charged by a server's byte
 * budget: its channel LLRs, information words and status, its work-area
 * entries, and the decoder state of its largest list stage (the LDS
 * footprint of that stage's layout, plus any part of it kept in global
 * memory). */
int polar_plan_frame_bytes(polar_plan p, uint64_t *bytes);

/* Admit one batch: frames [first, first + count) of d_frames, decoded as by
 * polar_scl_decode_batch with schedule 0 (outputs at the descriptors' out_off
 * in d_info, statuses at d_status[first ..]).  h_plan_idx (nullable) is a
 * host copy of the batch's plan indices (count entries, those of
 * d_frames[first ..]) used to charge the byte budget; without it every frame
 * is charged the most of the plan list.  Returns POLAR_OK and *slot, or
 * POLAR_EAGAIN when no slot is free or the budget cannot take the batch
 * (nothing enqueued), POLAR_EINVAL when count exceeds max_batch.  The call
 * allocates no device memory.  `tag` is returned by poll. */
int polar_server_submit(polar_server s, const polar_plan *plans, uint32_t n_plans,
                        const polar_frame *d_frames, uint32_t first, uint32_t count,
                        const uint32_t *h_plan_idx, const void *d_llr, uint32_t *d_info,
                        polar_status *d_status, uint64_t tag, uint32_t *slot);

/* Non-blocking: the tags of batches that completed since the last poll
 * (up to max), their slots freed.  *n receives the count. */
int polar_server_poll(polar_server s, uint64_t *tags, uint32_t max, uint32_t *n);

/* Frames admitted and not yet reported complete. */
int polar_server_inflight(polar_server s, uint32_t *frames);

int polar_server_destroy(polar_server s);

/* Serving session over requests pre-staged in device memory: request r is
 * frame r of d_frames and arrives at host time arrival_us[r] (microseconds
 * after the call starts, non-decreasing); h_plan_of (nullable) holds their
 * plan indices on the host, for the byte budget.  The loop releases
 * requests at their arrival times and, whenever a slot and budget are free,
 * admits the released requests not yet admitted (up to max_batch, and as
 * many as the budget takes) as one batch; it polls completions and writes,
 * per request, the host-observed completion time (us, same clock) to
 * complete_us.  stats (nullable, 5 values): batches, mean frames per batch,
 * largest frames in flight, session length in us, largest bytes in flight. */
int polar_serve_replay(polar_server s, const polar_plan *plans, uint32_t n_plans,
                       const polar_frame *d_frames, uint32_t n_req, const double *arrival_us,
                       const uint32_t *h_plan_of, const void *d_llr, uint32_t *d_info,
                       polar_status *d_status, double *complete_us, double *stats);

/* --------------------------------------------------------------- misc */
/* Frequency of the device realtime counter used by d_times, in kHz, for the
 * current device. */
int polar_device_clock_khz(uint32_t *khz);

const char *polar_strerror(int err);

/* Library version string. */
const char *polar_version(void);

#ifdef __cplusplus
}
#endif

#endif /* POLAR_SCL_H */
