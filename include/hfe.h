/*
 * hfe.h -- C ABI of the MI355X encrypted-CCMM library for private 1:N iris matching.
 *
 * The library implements the hot path of the paper "Private Iris Recognition with
 * High-Performance FHE" (arXiv 2601.17561): the RGSW-style encrypted matrix product
 * (CCMM, Section 2.3; database representation, Section 6.3) between an encrypted database
 * of masked ternary iris codes and a batch of encrypted query codes, with the key
 * generation, encryption, rescale (Section 2.2.4), decryption (Section 2.2.2) and
 * plaintext decision (equation (2), Section 2.1.3) around it.
 *
 * Conventions
 *  - Every function returns hfe_status (0 = HFE_OK, negative = error) and never throws or
 *    aborts.  After an error, hfe_last_error() returns a message (per thread).
 *  - Array arguments are DEVICE pointers (GPU memory of the current HIP device) unless the
 *    comment says "host".  Input arrays are borrowed: they must stay valid until the work
 *    enqueued on `stream` has passed the call.  Outputs are written by work enqueued on
 *    `stream`; synchronise the stream before reading them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All GPU work of a
 *    call is enqueued on that stream; validation errors return before anything is enqueued.
 *  - Handles (hfe_keys, hfe_db, hfe_qct, hfe_rct) are owned by the library and released with
 *    hfe_free().  A database or query handle refers to its keys: keep the keys alive while
 *    they are used.  Keys and databases are immutable once built and may be shared across
 *    threads; query and result handles are single-owner.
 *  - Device memory comes from the allocator installed with hfe_set_allocator(), else from
 *    hipMalloc / hipFree.
 *
 * Layouts (row-major unless stated; "residue" = uint64 in [0, prime))
 *  - Ternary matrices: int8 in {-1, 0, 1}.  M_DB: d1 x d2, one database code per row.
 *    M_Q: d3 x d2, one query vector per row (the paper's M_Q is its transpose).  The encryption
 *    calls check the entries on the device and return HFE_EINVAL for any other value (they wait
 *    for that check: the call returns after the work queued before it on the stream).
 *  - Primes: the database carries query primes q_0..q_{L-1} and one special prime p.
 *    A query of level l uses q_0..q_{l-1}; its scaling factor is
 *    Delta_l = 2^(floor(log2(q_0 ... q_{l-1})) - gap_bits).
 */
#ifndef HFE_H
#define HFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hfe_status;
enum {
  HFE_OK = 0,
  HFE_EINVAL = -1,     /* invalid argument or parameter (e.g. a prime != 1 mod 2N)      */
  HFE_ESHAPE = -2,     /* inconsistent sizes or row ranges                               */
  HFE_ELEVEL = -3,     /* level above the primes the database carries                    */
  HFE_ENOMEM = -4,     /* device allocation failed                                       */
  HFE_EDEVICE = -5,    /* HIP runtime error                                              */
  HFE_EBUSY = -6,      /* resource temporarily unavailable                               */
  HFE_EOVERFLOW = -7,  /* a bound needed for exact arithmetic does not hold              */
  HFE_EINTERNAL = -8
};

/* Contraction forms of hfe_ccmm (Section 6.3: the products mod Q reduced to small-integer
 * matrix products).  PLAIN_U64: 36-bit residues multiplied on the vector ALU with 128-bit
 * accumulation.  I8_MFMA: each centered residue split into 5 signed 8-bit digits, 25
 * digit-pair int8 MFMA products with int32 accumulation, exact recombination mod prime.
 * RNS_I8: the RNS technique of Section 6.3 applied per prime: each centered residue kept as its
 * balanced residues modulo n pairwise coprime moduli <= 256 (n = 11 for 36-bit primes and K up
 * to about 33,000; the product of the moduli is at least four times the largest exact sum), one int8
 * MFMA product per modulus with int32 accumulation (K < 2^17), then the Chinese remainder
 * reconstruction of the exact sum and its reduction mod the prime.
 * P2_I8: the n^2 technique of Section 6.3 applied per prime: for bases n_j among the primes
 * 211 <= n <= 251 (6 for 36-bit primes and K up to about 65,000; the product of the n_j^2 is at
 * least four times the largest exact sum), each centered residue's residue mod n_j^2 written as
 * M + n_j M' with |M|, |M'| <= 125; per base the three int8 MFMA products M N, M N' and M' N with
 * int32 accumulation (K <= 2^16) give the exact sum mod n_j^2, then the Chinese remainder
 * reconstruction and the reduction mod the prime.
 * All forms give the same residues.  The database stores 8, 5, n and 2 n bytes per entry and
 * prime for the four forms. */
typedef enum { HFE_FORM_PLAIN_U64 = 1, HFE_FORM_I8_MFMA = 2, HFE_FORM_RNS_I8 = 4, HFE_FORM_P2_I8 = 8 } hfe_form;

#define HFE_MAX_QPRIMES 8

typedef struct {
  uint32_t log_n_db;              /* N_DB = 2^log_n_db, database ring degree, 1..16 (up  */
                                  /* to 2^14 one LDS-resident transform per polynomial,  */
                                  /* 2^15 and 2^16 two passes through device memory)     */
  uint32_t log_n_q;               /* N_Q = 2^log_n_q, query ring degree, 1..16           */
  uint32_t n_q_primes;            /* L, query primes carried by the database, 1..8       */
  uint64_t q[HFE_MAX_QPRIMES];    /* q_0..q_{L-1}: distinct primes < 2^36, = 1 mod 2N    */
  uint64_t p;                     /* special prime < 2^36, = 1 mod 2N, distinct from q_i */
  uint32_t gap_bits;              /* Delta_l = 2^(floor(log2 Q_l) - gap_bits)            */
  uint32_t d2;                    /* code length (columns of M_DB)                       */
  uint32_t max_db_rows;           /* largest d1 the keys cover: ceil(max/N_DB) secrets   */
  uint32_t t_num, t_den;          /* match threshold t = t_num / t_den, 0 < t < 1/2      */
} hfe_params;

typedef struct hfe_keys hfe_keys;  /* secrets and per-prime NTT tables                   */
typedef struct hfe_db hfe_db;      /* encrypted database, resident on the device         */
typedef struct hfe_qct hfe_qct;    /* encrypted query batch                              */
typedef struct hfe_rct hfe_rct;    /* encrypted CCMM result                              */

/* Device allocator hook: alloc(bytes, stream, ctx) returns device memory usable in stream
 * order on `stream` (NULL on failure), aligned to at least 256 bytes as hipMalloc's is (the
 * kernels read and write 16-byte vectors at offsets that are multiples of 16 from the start);
 * dealloc(ptr, stream, ctx) releases it in stream order.  Passing NULL functions restores
 * hipMalloc / hipFree. */
typedef void* (*hfe_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*hfe_dealloc_fn)(void* ptr, void* stream, void* ctx);
hfe_status hfe_set_allocator(hfe_alloc_fn alloc, hfe_dealloc_fn dealloc, void* ctx);

/* Fill *out (host) with default parameters: the largest primes < 2^36 that are = 1 mod 2^17
 * (the first is p, the next n_q_primes are q_0..), gap 20, threshold 3/8. */
hfe_status hfe_default_params(uint32_t log_n_db, uint32_t log_n_q, uint32_t n_q_primes,
                              uint32_t d2, uint32_t max_db_rows, hfe_params* out);

/* Key generation (Section 2.2.2, single key holder): ternary query secrets s_j in R_{N_Q},
 * j < ceil(d2/N_Q), and database secrets s'_j in R_{N_DB}, j < ceil(max_db_rows/N_DB),
 * drawn from the Philox4x64-10 streams keyed by `seed`.  Synchronous. */
hfe_status hfe_keygen(const hfe_params* params, uint64_t seed, hfe_keys** out);

/* The paper's own modulus chain (Section 6.3, "Fast PPMM using int8 cuBLAS"): the ciphertext
 * modulus is a product of squares n^2 of primes 127 <= n <= 253, so a product modulo it is a product
 * modulo each n^2, three int8 MFMA products of the digits M + n M' (|M|, |M'| <= 126), with no exact
 * integer to rebuild.  Query modulus Q_l = n_0^2 ... n_{l-1}^2 (l <= n_q_mods); special part
 * P = the product of the next n_p_mods squares, the database scale and the rescale divisor
 * (RS_P(x) = floor(x / P + 1/2) mod Q_l; P odd); database modulus Q P.  The secrets, the ring degrees
 * and the scale Delta_l = 2^(floor(log2 Q_l) - gap_bits) are as for the prime family; products with
 * the ternary secrets are exact integers (at most N n^2 / 2 in magnitude) computed through the NTT
 * modulo ntt_prime.  Keys from hfe_chain_keygen work with hfe_encrypt_db (forms HFE_FORM_P2_I8, plus
 * HFE_FORM_PLAIN_U64 to keep the residues for hfe_export: [modulus: query bases, then the special
 * part's][column][row], each mod its n^2), hfe_encrypt, hfe_ccmm and hfe_ccmm_noalloc (form
 * HFE_FORM_P2_I8; needs d2 + N_Q <= 2^16), hfe_ccmm_product (C: (level + n_p_mods) x d3 x (N_DB + rows)
 * residues, the level's query moduli then the special ones), hfe_decrypt, hfe_match, hfe_export and
 * hfe_shape; batches, plans, the server, the autotuner and database files refuse them (HFE_EINVAL).
 * Result residues are mod n_j^2 in the order [j < level][column][A_out | B_out]. */
#define HFE_CHAIN_MAX_BASES 11
typedef struct {
  uint32_t log_n_db, log_n_q;       /* ring degrees, 1..16 each                                  */
  uint32_t n_q_mods;                /* query moduli, 1..8                                        */
  uint32_t n_p_mods;                /* special moduli, 1..3                                      */
  uint32_t bases[HFE_CHAIN_MAX_BASES]; /* n: the query bases, then the special part's; distinct  */
                                    /* primes in [127, 253]                                      */
  uint64_t ntt_prime;               /* prime < 2^36, = 1 mod 2N, for the secret products         */
  uint32_t gap_bits;                /* Delta_l = 2^(floor(log2 Q_l) - gap_bits)                  */
  uint32_t d2, max_db_rows;         /* code length; largest d1 the keys cover                    */
  uint32_t t_num, t_den;            /* match threshold                                           */
} hfe_chain_params;
/* Defaults: the largest primes of the range first (query bases), the next ones for P; ntt_prime
 * the largest prime < 2^36 that is 1 mod 2^17; gap 20; threshold 3/8. */
hfe_status hfe_chain_default_params(uint32_t log_n_db, uint32_t log_n_q, uint32_t n_q_mods, uint32_t n_p_mods,
                                    uint32_t d2, uint32_t max_db_rows, hfe_chain_params* out);
/* Key generation for the chain: the same ternary secrets as hfe_keygen with the same seed.
 * HFE_EINVAL for parameters outside the ranges above; HFE_EOVERFLOW as hfe_keygen for d2 against
 * gap_bits.  A level whose Q_l has fewer than gap_bits + 2 bits is refused by hfe_encrypt
 * (HFE_ELEVEL). */
hfe_status hfe_chain_keygen(const hfe_chain_params* params, uint64_t seed, hfe_keys** out);

/* Masked ternary encoding (Section 2.1.3) with cyclic shifts (Section 2.1.2):
 * out[(e * n_shifts + s) * d2 + t] = m' - 2 (c' AND m') with c' = code row e and m' = mask
 * row e, both rolled by shifts[s] (rolled[t] = x[(t - shifts[s]) mod d2]).
 * codes, masks: n x d2 uint8 in {0,1}; shifts: host array of n_shifts int32;
 * out: (n * n_shifts) x d2 int8. */
hfe_status hfe_encode(const uint8_t* codes, const uint8_t* masks, int64_t n, int32_t d2,
                      const int32_t* shifts, int32_t n_shifts, int8_t* out, void* stream);

/* Database encryption in the RGSW/MSRLWE form of Sections 2.3 and 6.3: T = M_DB S_Q, and per
 * prime of Q_L p: A = [A1 | A2] uniform (N_DB x (d2 + N_Q)), B = -S_DB A + p [M_DB | T] + E.
 * m_db: d1 x d2 ternary (device).  forms: bitmask of hfe_form the database is prepared for
 * (HFE_FORM_RNS_I8 needs d2 + N_Q < 2^17 and HFE_FORM_P2_I8 d2 + N_Q <= 2^16, else HFE_ESHAPE).
 * The result stays resident on the device. */
hfe_status hfe_encrypt_db(const hfe_keys* keys, const int8_t* m_db, int64_t d1, uint64_t seed,
                          uint32_t forms, void* stream, hfe_db** out);

/* The encrypted database is the artefact prepared once and kept (Section 6.3: it is stored and
 * stays resident, and its size is the scheme's main storage cost), so it can be written to a file
 * and read back instead of being encrypted again.
 * hfe_db_save: writes `db` (every form it was prepared for) to the file `path` (host path; created
 *   or truncated), after the work already queued on `stream`.  Synchronous: the file is complete
 *   when the call returns.  Host memory used: a 64 MiB pinned staging buffer.
 * hfe_db_load: reads a file written by hfe_db_save under the same keys (parameters and secrets,
 *   checked by a fingerprint) into a new resident database holding the forms in `forms` (a subset
 *   of the file's; 0: all of them; the others' bytes are skipped); `stream` orders the copies,
 *   and the data is on the device when the call returns.  Release the result with hfe_free.
 * Errors: HFE_EINVAL for an invalid handle, a NULL path, a file that cannot be opened or written,
 * one that is not a database file of this library version, was written under other keys, lacks a
 * requested form, or is truncated or longer than its header says; HFE_ENOMEM / HFE_EDEVICE from
 * the device. */
hfe_status hfe_db_save(const hfe_db* db, const char* path, void* stream);
/* Device bytes the database holds for one form (0: all its forms): the planes of Section 6.3's
 * storage count, (N_DB + d1) (d2 + N_Q) entries per prime times 8 bytes (plain), 5 (digits),
 * n (RNS) or 2 n (n^2), in their padded layouts (K rounded up to 64, rows to 64 plus 256). */
hfe_status hfe_db_bytes(const hfe_db* db, uint32_t form, size_t* bytes);
hfe_status hfe_db_load(const hfe_keys* keys, const char* path, uint32_t forms, void* stream, hfe_db** out);

/* Query encryption in MSRLWE form (Section 2.3): per column c and query prime,
 * a_c uniform in R_{N_Q}, b_c = -S_Q a_c + Delta_level m_c + e_c (chunks of N_Q rows share
 * a_c, each under its own secret).  m_q: d3 x d2 ternary (device); 1 <= level <= L. */
hfe_status hfe_encrypt(const hfe_keys* keys, const int8_t* m_q, int64_t d3, uint32_t level,
                       uint64_t seed, void* stream, hfe_qct** out);

/* The encrypted matrix product (Section 2.3, the four plaintext products written as one
 * product per prime; Section 6.3): lift the query residues from Q to Q p (centered),
 * C = D X mod prime for the level's primes and p, then rescale by p
 * (Section 2.2.4, RS_p(x) = floor(x/p + 1/2) mod Q).  The database rows used are the
 * N_DB A-part rows and the database codes [row0, row0 + rows).  form: hfe_form. */
hfe_status hfe_ccmm(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t form,
                    void* stream, hfe_rct** out);

/* The exact product before the rescale, for parity checks of the contraction: the lift and the
 * contraction of hfe_ccmm in form `form`, without RS_p.  C (device, (level + 1) x d3 x (N_DB + rows)
 * uint64, caller-owned) receives C[z][c][r] = sum_k D[src(r)][k] L(x_c)[k] mod prime_z for the
 * level's primes z < level and p (z = level), where L is the centered lift of query column c and
 * row r < N_DB is A-part row r, row N_DB + i database code row0 + i.  The small-modulus forms
 * reconstruct these residues with their reconstruction kernel alone (hfe_ccmm fuses it with the
 * rescale).  Errors as hfe_ccmm; C NULL: HFE_EINVAL. */
hfe_status hfe_ccmm_product(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t form,
                            void* stream, uint64_t* C);

/* Allocation-free CCMM, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same lift, contraction and
 * rescale as hfe_ccmm, in any form, with the same results, but the call's device buffers (query
 * planes, the contraction output or the small-modulus residues) come from a static device array
 * of HFE_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the process
 * ends, and the result goes to caller memory.  No hipMalloc, hipFree or allocator call is made.
 *   out: device, level x d3 x (N_DB + rows) uint64 (caller-owned), receives the rescaled residues
 *        in the order of hfe_export(rct, 0): [prime < level][column][A_out (N_DB) | B_out (rows)].
 * Errors: those of hfe_ccmm; out NULL: HFE_EINVAL; a call whose buffers exceed the array (e.g. more
 * than about 128 query columns of the digit form, or 16 of the RNS form, against a database of
 * K = 20,992 and 30,720 rows at three query primes plus p): HFE_ENOMEM with nothing enqueued;
 * HFE_EDEVICE if the array's address cannot be resolved.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams or host threads) race on it and must be ordered by the caller.  Nothing in the array
 * needs clearing between calls (each call writes every byte it reads).
 * hfe_noalloc_init: resolves the array's address on the current device ahead of the first call
 * (optional; the first call on a device does it otherwise). */
#define HFE_NOALLOC_SCRATCH_BYTES (256ull << 20)
hfe_status hfe_noalloc_init(void);
hfe_status hfe_ccmm_noalloc(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t form,
                            uint64_t* out, void* stream);

/* An empty result handle shaped for query q against every code of db (level x d3 x (N_DB + d1)
 * residues, allocated on `stream`), for hfe_server_submit_encrypted.  Release with hfe_free. */
hfe_status hfe_result_create(const hfe_db* db, const hfe_qct* q, void* stream, hfe_rct** out);

/* Batched CCMM: item i is its own CCMM of items[i].q (any level, any column count) against the
 * database codes [items[i].row0, items[i].row0 + items[i].rows), all against one database.
 * Items with the same level and row range form one problem, their query columns side by side (so
 * only a problem pads its columns to whole tiles); a level whose items cover several row ranges is
 * split into one problem over the N_DB A rows for all its columns and one problem per row range
 * over that range's rows.  int8 forms (HFE_FORM_I8_MFMA, HFE_FORM_RNS_I8, HFE_FORM_P2_I8):
 * one grouped launch lifts and splits every item's query, ONE persistent launch computes the tiles
 * of every problem, prime (and small modulus or base) (workgroups claim tiles of a device-resident
 * tile table in order), for the RNS and n^2 forms one grouped launch reconstructs the residues mod
 * each prime,
 * and one grouped launch rescales every item; the digit form's problems share one tile
 * configuration (the forced one, else of the tuned and the default configuration the one that pads
 * the problems least); plain form: one hfe_ccmm per item.  outs[i] receives item i's result handle
 * (release each with hfe_free).  1 <= n <= 256. */
typedef struct {
  const hfe_qct* q;
  int64_t row0, rows;
} hfe_batch_item;
hfe_status hfe_ccmm_batched(const hfe_db* db, const hfe_batch_item* items, int32_t n, int32_t form,
                            void* stream, hfe_rct** outs);

/* Reusable batched int8 CCMM for repeated batches (e.g. serving steps), in the int8 form `form`
 * (HFE_FORM_I8_MFMA, HFE_FORM_RNS_I8 or HFE_FORM_P2_I8, prepared in the database): the workspace
 * for up to max_items items, max_cols query columns in total and levels up to max_level is
 * allocated once;
 * hfe_plan_run writes the batch's descriptor tables (a host-to-device copy on `stream`) and
 * enqueues the grouped launches; with use_graph they are captured, on the first run that uses a
 * tile configuration, into a hipGraph that later runs with that configuration replay (any later
 * stream is fine; the graph is launched on it).  hfe_plan_result
 * returns item i's result of the last run as a view owned by the plan: valid until the next
 * hfe_plan_run or hfe_free(plan); hfe_free on the view does nothing.  Runs on one plan must not
 * overlap; the plan's database must outlive it. */
typedef struct hfe_plan hfe_plan;
hfe_status hfe_plan_create(const hfe_db* db, int32_t max_items, int64_t max_cols, uint32_t max_level,
                           int32_t form, hfe_plan** out);
/* hfe_plan_create_for: a plan whose workspace is sized exactly for the batch `items` (n items):
 * the query planes, contraction output, residues and results that batch needs, rather than the
 * worst case of a column count and level over the whole database.  It runs that batch and any
 * batch of at most n items whose needs fit every one of those capacities (else hfe_plan_run
 * returns HFE_ESHAPE).  Errors as hfe_plan_create and hfe_ccmm_batched's item checks. */
hfe_status hfe_plan_create_for(const hfe_db* db, const hfe_batch_item* items, int32_t n, int32_t form,
                               hfe_plan** out);
hfe_status hfe_plan_run(hfe_plan* plan, const hfe_batch_item* items, int32_t n, int32_t use_graph,
                        void* stream);
hfe_status hfe_plan_result(const hfe_plan* plan, int32_t i, const hfe_rct** view);

/* Autotuner of the int8 contraction tiles: times every tile configuration (see hfe_i8_variants)
 * on this problem (one untimed run each, then reps rounds that time every configuration once,
 * keeping each configuration's best), records the fastest for the
 * problem's (level, query-column bucket; buckets are powers of two from 64) and returns it in
 * *best.  Later hfe_ccmm calls, batches (by their largest level and mean column count) and plans
 * (at creation) use the entry of their level with the nearest bucket, else the default.  The
 * table can be saved and loaded as text ("<level> <column bucket> <configuration name>" per
 * line). */
hfe_status hfe_autotune(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t reps,
                        void* stream, int32_t* best);
hfe_status hfe_autotune_save(const char* path);
hfe_status hfe_autotune_load(const char* path);

/* Continuous-batching server over a resident database, in the int8 form `form` (HFE_FORM_I8_MFMA,
 * HFE_FORM_RNS_I8 or HFE_FORM_P2_I8, prepared in the database).  A worker thread keeps
 * n_slots steps in flight on their own streams; each step admits queued requests in arrival
 * order while their columns fit the step (at most max_cols_per_step columns, at most
 * max_items_per_step requests, and the memory budget: mem_budget bytes of workspace split over
 * the slots, allocated at creation), runs them as one batched CCMM (captured hipGraph) and
 * decrypts every request into its own output.  Requests that arrive while steps run are
 * admitted by the next free slot, so their work overlaps on the device.  A request larger than
 * one step is rejected (HFE_EBUSY).  All device memory is allocated by hfe_server_create; the
 * worker allocates nothing.
 *   hfe_server_submit: q (its keys must be the server's; level <= max_level) stays borrowed
 *     until the ticket completes; ip_out: device int32 d3 x d1 (query-major) receives the
 *     decrypted inner products against every database code.
 *   hfe_server_submit_encrypted: the same, but the request's encrypted result (the rescaled
 *     residues against every database code, as hfe_ccmm returns them) is copied into `result`,
 *     a handle from hfe_result_create for this query, which stays borrowed until the ticket
 *     completes; the key holder decrypts it with hfe_decrypt afterwards.  The server then needs
 *     no secret for that request.
 *   hfe_server_poll: *state = 0 queued, 1 running, 2 done, or a negative status: HFE_EBUSY
 *     (rejected as larger than one step, or still queued when the server was freed), another
 *     status (its step failed).
 *   hfe_server_wait: blocks until the ticket is done (HFE_OK) or failed (its negative status),
 *     at most timeout_ms (< 0: no limit; then HFE_EBUSY, and hfe_server_poll tells a timeout,
 *     state 0 or 1, from a rejection).
 *   hfe_server_drain: blocks until no request is queued and no step runs (HFE_OK), at most
 *     timeout_ms (< 0: no limit; then HFE_EBUSY).  Every ticket submitted before the call has
 *     then finished, including those already beyond the retention window below.
 *   hfe_server_stats: counts and latencies (arrival -> result ready; admission -> ready) of the
 *     requests completed since creation or the last reset: percentiles over the most recent
 *     65,536 completions, the mean over all of them.  retained: request records the server
 *     holds (queued, running, and the last 1,024 finished); max_busy_slots: the most slots
 *     that held a step at once; overlap_pairs: pairs of steps on different slots whose device
 *     intervals (timing events around each step on its stream) intersected.
 *   hfe_server_reset_stats: clears the statistics and forgets finished requests (their tickets
 *     become unknown).  Without resets the server keeps the records of the last 1,024 finished
 *     tickets (older ones become unknown to poll and wait), so its host memory stays bounded. */
typedef struct hfe_server hfe_server;
typedef struct {
  int64_t submitted, completed, rejected, steps, max_queue;
  double p50_ms, p99_ms, service_p50_ms, service_p99_ms, mean_ms;
  double req_per_s, cmp_per_s, mean_cols_per_step, elapsed_s;
  int64_t retained, max_busy_slots, overlap_pairs;
} hfe_server_report;
hfe_status hfe_server_create(const hfe_db* db, size_t mem_budget, int64_t max_cols_per_step,
                             int32_t max_items_per_step, int32_t n_slots, uint32_t max_level, int32_t form,
                             hfe_server** out);
hfe_status hfe_server_submit(hfe_server* srv, const hfe_qct* q, int32_t* ip_out, uint64_t* ticket);
hfe_status hfe_server_submit_encrypted(hfe_server* srv, const hfe_qct* q, hfe_rct* result, uint64_t* ticket);
hfe_status hfe_server_poll(hfe_server* srv, uint64_t ticket, int32_t* state);
hfe_status hfe_server_wait(hfe_server* srv, uint64_t ticket, int64_t timeout_ms);
hfe_status hfe_server_drain(hfe_server* srv, int64_t timeout_ms);
hfe_status hfe_server_stats(hfe_server* srv, hfe_server_report* out);
hfe_status hfe_server_reset_stats(hfe_server* srv);

/* Decryption and coefficient decoding (Sections 2.2.1, 2.2.2): for column c and code r,
 * y = B_out + (s'_j * A_out)[r mod N_DB] mod Q (CRT over the level's primes, centered),
 * v[c * rows + r] = y / Delta (double) and ip[c * rows + r] = floor(y / Delta + 1/2).
 * v may be NULL.  v, ip: d3 x rows (device). */
hfe_status hfe_decrypt(const hfe_keys* keys, const hfe_rct* r, double* v, int32_t* ip,
                       void* stream);

/* Plaintext decision (equation (2)): score = ip / popcount(m_q AND m_db) > 1 - 2t, decided in
 * integers as ip * t_den > (t_den - 2 t_num) * overlap (no match without overlap).
 * ip: d3 x rows int32 (d3 = n_eyes * n_shifts, eye-major as produced by hfe_encode);
 * q_masks: n_eyes x d2 uint8 (unshifted); db_masks: rows x d2 uint8 (the rows ip covers);
 * shifts: host, n_shifts int32.  Outputs: decision d3 x rows uint8 (may be NULL),
 * eye_match n_eyes uint8 = OR over the eye's shifts and all rows. */
hfe_status hfe_match(const int32_t* ip, const uint8_t* q_masks, int64_t n_eyes,
                     const int32_t* shifts, int32_t n_shifts, const uint8_t* db_masks,
                     int64_t rows, int32_t d2, uint32_t t_num, uint32_t t_den,
                     uint8_t* decision, uint8_t* eye_match, void* stream);

/* Export residues to host memory for parity checks (synchronous: waits for the device).
 * `which` selects an array; elements [offset, offset + n) of its canonical order are copied
 * to the host array dst.  Canonical orders:
 *   keys  0: query secrets    [j < k][t < N_Q]      (int64 two's complement in uint64)
 *         1: database secrets [j < k'][t < N_DB]
 *   db    0: D per prime, column-major: [prime (q_0..q_{L-1}, p)][col < d2 + N_Q][row < N_DB + d1]
 *            (available when the database was prepared for HFE_FORM_PLAIN_U64)
 *   qct   0: query            [prime < level][column < d3][b_c (d2) | a_c (N_Q)]
 *   rct   0: result           [prime < level][column < d3][A_out (N_DB) | B_out (rows)]
 * If dst is NULL, *count receives the total number of elements and nothing is copied. */
hfe_status hfe_export(const void* handle, int32_t which, size_t offset, uint64_t* dst, size_t n,
                      size_t* count);

/* ---------------------------------------------------------------- FormatSwitch (Appendix C.1)
 * The query reaches the CCMM from a transmission ring R_{N_T} (N_T = 2^16 in the paper): RLWE
 * ciphertexts (a, b) modulo Q' = q_0 .. q_l under a transmission secret s_T, one per chunk j of
 * N_Q code positions of a query column c (ciphertext col = c k + j), the chunk's entries m at the
 * coefficients of degree divisible by rho = N_T / N_Q:  b = -a s_T + (Delta_l q_l) m~ + e.
 * FormatSwitch turns them into the query ciphertext of level l that hfe_ccmm takes: a key switch
 * from s_T to s'(X^rho) (one digit [a (Q'/q_i)^-1]_{q_i} per prime, keys modulo Q' p, rescale by
 * p) followed by the extraction of the coefficients of degree divisible by rho (the trace: a
 * ciphertext under s' in R_{N_Q}), the conversion of the k chunks of a column to the MSRLWE format
 * under the CCMM secrets s_0 .. s_{k-1} (conversion keys whose masks are shared by the k outputs,
 * rescale by p), and the modulus switch from Q' to q_0 .. q_{l-1} (rescale by q_l), which brings
 * the scale from Delta_l q_l to Delta_l.
 * Transmission layout T (uint64 residues): [prime i <= l][col < d3 k][a | b][t < N_T]. */
typedef struct hfe_fskeys hfe_fskeys;

/* FormatSwitch keys for queries of level `level` (1 <= level < n_q_primes of `keys`: the
 * transmission modulus takes one prime more) from ring degree 2^log_n_t (log_n_q <= log_n_t <= 16):
 * s_T, s' and the ring-switching and conversion keys, drawn from `seed` (streams of their own).
 * Needs keys of the prime family with 6 <= log_n_q <= 14; keeps a reference to `keys` (keep them
 * alive).  hfe_export(fskeys, 0 | 1) gives s_T (N_T) | s' (N_Q); hfe_shape gives {level,
 * log_n_t, rho, k}.  Device memory: about 2 (level + 1) (level + 2) N_T doubles of keys. */
hfe_status hfe_fs_keygen(const hfe_keys* keys, uint32_t level, uint32_t log_n_t, uint64_t seed, hfe_fskeys** out);

/* Number of uint64 in the transmission ciphertexts of d3 query columns: (level+1) d3 k 2 N_T. */
hfe_status hfe_fs_transmit_count(const hfe_fskeys* fk, int64_t d3, int64_t* count);

/* The client's transmission encryption of M_Q (d3 x d2 ternary, device) into T (device, the count
 * above), draws from `seed`.  Uses a workspace of d3 k (level + 1) N_T doubles.  HFE_EINVAL for
 * entries outside {-1, 0, 1} (the call waits for that check). */
hfe_status hfe_fs_encrypt(const hfe_fskeys* fk, const int8_t* m_q, int64_t d3, uint64_t seed, uint64_t* T,
                          void* stream);

/* FormatSwitch of the transmission ciphertexts T of d3 query columns (layout above, residues below
 * their primes; T is only read) into a query ciphertext of level `level` under the CCMM keys, for
 * hfe_ccmm.  Workspace: d3 k ((level + 1) N_T + 2 (level + 2) N_Q) + 3 (level + 2) d3 N_Q doubles
 * for k <= 2.  With hfe_profile(1) the query records its stage boundaries, read by
 * hfe_fs_profile_ms (0: digits, 1: ring switch, 2: conversion, 3: rescales and output). */
hfe_status hfe_format_switch(const hfe_fskeys* fk, const uint64_t* T, int64_t d3, void* stream, hfe_qct** out);
hfe_status hfe_fs_profile_ms(const hfe_qct* q, float* ms, int32_t n);

/* ---------------------------------------------------------------- normalise and fold
 * The step after the CCMM in Algorithm 2 (Section 4.1-4.3, Appendix C.2): a block of rho score
 * ciphertexts ct_c, c < rho (slot j of ct_c holds the inner product of query column c with database
 * entry j), becomes ceil(rho / k) ciphertexts
 *   ct'_r = sum_{r' < min(k, rho - r k)} Rot_{r k + r'}( f( ct_{r k + r'} (.) Ecd(1 / count_{r k + r'}) ) )
 * where count_c[j] = ||m_q,c AND m_db,j||_1 normalises the inner products into scores (a plaintext
 * product), f is the degree-7 folding polynomial of Appendix C.2, evaluated in three levels, and Rot_r
 * moves slot i to slot i + r (Section 4.3: slot i of the result holds the score of entry i - r).
 * CKKS at ring degree N = 2^log_n (N/2 real slots, slot j at the root zeta^(5^j mod 2N)), secret of
 * Hamming weight 32, moduli q_0 (36 bits), q_1 .. q_3 (near 2^23: the three levels of f at the scale of
 * Appendix C.2), q_4 (36 bits: the normalisation) and a special prime p (36 bits) for key switching
 * (one digit per prime).  Inputs are encrypted at scale 2^20 at level 4; the rotations and the sums of
 * a group run at level 1 before one last rescale; folded ciphertexts sit at level 0 with scale 2^24.
 * Rot_{r k + r'} is applied as Rot_{r k} after Rot_{r'}.  Ciphertexts live on the device in the NTT domain; hfe_export(fct, 0)
 * gives their coefficient residues [count][b | a][q_0 .. q_level][N], hfe_shape(fct) {level, count,
 * N, scale}, hfe_export(foldkeys, 0) the secret (N coefficients), hfe_shape(foldkeys) {log_n, k,
 * rho, rotation keys}. */
typedef struct hfe_foldkeys hfe_foldkeys;
typedef struct hfe_fct hfe_fct;

/* Keys for folds with factor k of blocks of at most rho ciphertexts (6 <= log_n <= 14, 1 <= k, rho
 * <= N/2): the secret, relinearisation keys at levels 1 .. 3 and rotation keys (level 1) for the
 * amounts 1 .. min(k, rho) - 1 and r k (1 <= r < ceil(rho / k)), drawn from `seed`.  Device memory:
 * about (68 + 13 (keys of rotation)) N doubles. */
hfe_status hfe_fold_keygen(uint32_t log_n, uint32_t k, uint32_t rho, uint64_t seed, hfe_foldkeys** out);

/* Encryption of `count` vectors of N/2 inner products (device int32, [count][N/2], each in
 * -2^24 .. 2^24) at scale 2^10 and level 4, draws from `seed`.  HFE_EINVAL for a value out of range
 * (the call waits for that check). */
hfe_status hfe_fold_encrypt(const hfe_foldkeys* fk, const int32_t* ip, int64_t count, uint64_t seed, void* stream,
                            hfe_fct** out);

/* The fold of the ciphertexts `in` (level 4, count a multiple of rho, rho at most the keys' rho) in
 * blocks of rho, with the mask counts (device int32, [count][N/2], each in 1 .. 2^24; the call waits
 * for that check): count / rho * ceil(rho / k) ciphertexts at level 0, block-major.  Workspace: about
 * 14 count N uint64.  With hfe_profile(1) the result records its stage boundaries, read by
 * hfe_fold_profile_ms (0: the normalisation plaintexts, 1: normalisation, 2: f, 3: rotations and sums). */
hfe_status hfe_fold(const hfe_foldkeys* fk, const hfe_fct* in, const int32_t* counts, int64_t rho, void* stream,
                    hfe_fct** out);
hfe_status hfe_fold_profile_ms(const hfe_fct* ct, float* ms, int32_t n);

/* Decryption and decoding of folded ciphertexts (level 0) into values (device doubles,
 * [count][N/2]): the real parts of the slots divided by the scale. */
hfe_status hfe_fold_decrypt(const hfe_foldkeys* fk, const hfe_fct* ct, double* values, void* stream);

/* Shape queries of a handle (host): dims[0..3] = {level or L, d3 or d1, rows, K}. */
hfe_status hfe_shape(const void* handle, int64_t* dims);

/* Stage timing for measurement.  hfe_profile(1) makes later hfe_ccmm calls record HIP events on
 * their stream around each stage (0: lift and digit split, 1: contraction kernel, 2: rescale);
 * hfe_profile_ms(result, ms, n) waits for those events and writes the first n (<= 3) stage
 * durations in milliseconds to host array ms.  HFE_EINVAL if the result was made without
 * profiling. */
hfe_status hfe_profile(int32_t enable);
hfe_status hfe_profile_ms(const hfe_rct* r, float* ms, int32_t n);

/* Rate probes: the instruction ceilings of the two contraction forms (Section 6.3's int8 matrix
 * products and the plain 64-bit residue products), measured on the current device.
 *   which = HFE_PROBE_MFMA_I8: int8 MFMA products (32 x 32 x 32) whose operands stream random
 *     bits, as the digit planes of ciphertexts do; *rate = int8 operations per second (two per
 *     multiply-add).
 *   HFE_PROBE_MFMA_I8_ZERO: the same products on all-zero operands (the issue ceiling).
 *   HFE_PROBE_VALU_MAD_U64: 32 x 32 -> 64-bit multiply-adds (v_mad_u64_u32) per second, lane
 *     operations; the plain form spends four per residue multiply-add.
 * iters >= 1: loop trips per wave of the timed launch (one untimed launch of iters / 8 + 1 trips
 * runs first).  The call allocates a small sink buffer, synchronises `stream` and returns the
 * rate of the timed launch (HIP events on `stream`).  HFE_EINVAL for another `which`. */
enum { HFE_PROBE_MFMA_I8 = 1, HFE_PROBE_MFMA_I8_ZERO = 2, HFE_PROBE_VALU_MAD_U64 = 3 };
hfe_status hfe_probe_rate(int32_t which, int64_t iters, void* stream, double* rate);

/* Tile configurations of the int8-MFMA contraction kernel.  hfe_i8_variants() returns their
 * number (configuration 0 is the default); hfe_i8_variant_name(v) names one (NULL if v is out of
 * range): "dma*" configurations load the digit planes straight into LDS ("q128" / "r128": 128
 * query columns / database rows per workgroup, "w<n>": waves per SIMD), "pipe_w1" prefetches
 * through registers, "r<a>q<b>b<c>w<d>" are register-staged tiles of a x b waves with c LDS
 * buffers.  hfe_set_i8_variant(v) forces the configuration of later calls, overriding the
 * autotuner (-1 restores the default choice).  Every configuration computes the same residues. */
int32_t hfe_i8_variants(void);
const char* hfe_i8_variant_name(int32_t v);
hfe_status hfe_set_i8_variant(int32_t v);

/* Release any handle (NULL-safe).  Waits for work that uses it on its stream. */
void hfe_free(void* handle);

/* Message for the last non-OK status returned on this thread. */
const char* hfe_last_error(void);

/* The library's discrete-Gaussian table T[j] = floor(2^64 P(|e| <= j)), j < 19, computed on
 * the host in quad precision (sigma = 3.2, tail 19).  dst: host, 19 entries. */
hfe_status hfe_cdt_table(uint64_t* dst);

#ifdef __cplusplus
}
#endif

#endif /* HFE_H */
