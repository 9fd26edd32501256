/*
 * carve.h -- C ABI of the MI355X (gfx950) hash-based sector carving library.
 *
 * The method (Collange, Dandass, Daumas, Defour, "Using Graphics Processors
 * for Parallelizing Hash-based Data Carving"):
 *   - Section 2: a sector is 512 bytes and a cluster is 8 consecutive sectors;
 *     files of interest start on a cluster and occupy whole sectors.
 *   - Eq. (1), Section 2.2, with the 64-bit accumulator of Section 4: the
 *     signature of a sector is djb2, h = 5381, h = h*33 + s for each byte s
 *     (unsigned, address order), modulo 2^64.
 *   - Section 3.1: the signatures of the master ("known") sectors at cluster
 *     position tau form the set S_tau; a disk sector at position tau is
 *     flagged when its signature is in S_tau, and flagged sectors are
 *     confirmed by a byte-for-byte comparison with the master sectors of the
 *     same signature.
 *
 * Conventions for every entry point:
 *   - Return value: CARVE_OK (0) or a negative carve_status. On failure,
 *     carve_last_error() returns a message for the calling thread.
 *   - "device" pointers are HIP device memory of the current device (for
 *     example a torch tensor's data_ptr()); "host" pointers are host memory;
 *     "host or device" accepts either.
 *   - Byte buffers of sectors must be 16-byte aligned.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Sector ids are relative to the start of the buffer passed in.
 *   - Nothing here allocates or frees the caller's buffers.
 */
#ifndef CARVE_H
#define CARVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct carve_index carve_index; /* resident master-signature index */
typedef struct carve_scan carve_scan;   /* result buffers of one scan      */
typedef struct carve_batch carve_batch; /* result buffers of a batch scan  */

typedef enum {
  CARVE_OK = 0,
  CARVE_EINVAL = -1,       /* bad argument: null/misaligned pointer, bad enum, bad sizes */
  CARVE_ENOMEM = -2,       /* device or host allocation failed */
  CARVE_ETRUNC = -3,       /* output capacity too small; *n_out holds the full count */
  CARVE_EDEVICE = -4,      /* a HIP call failed */
  CARVE_EUNSUPPORTED = -5  /* valid request this build does not handle */
} carve_status;

typedef enum {
  CARVE_SIG_DJB2_64 = 0,   /* Eq. (1), 64-bit accumulator (Section 4) */
  CARVE_SIG_CRC64_ISO = 1  /* the 64-bit CRC of Section 2.1, read as CRC-64/GO-ISO: generator
                              x^64 + x^4 + x^3 + x + 1, reflected in and out, register preset to
                              all ones, result complemented (check value of "123456789":
                              0xb90956c775a41001) */
} carve_sig_kind;

typedef enum {
  CARVE_TAU_PER_CLUSTER = 0, /* sector j matches S_tau with tau = (j + tau0) mod 8 (Section 3.1) */
  CARVE_TAU_ANY = 1          /* sector j matches a master sector at any cluster position */
} carve_tau_mode;

/* How a scan looks a signature up (Section 3.2, Eq. (3), and the occupancy
 * study of Section 4). Every layout gives the same results. */
typedef enum {
  CARVE_LAYOUT_BUCKETED = 0, /* linear probing over 128-byte buckets of 16 keys, home bucket from a
                                multiplicative hash of the signature (the default) */
  CARVE_LAYOUT_LINEAR = 1,   /* the paper's table: home slot = the w low bits of the signature,
                                linear probing slot by slot (Eq. (3)) */
  CARVE_LAYOUT_SORTED = 2    /* the distinct signatures sorted, binary search */
} carve_index_layout;

typedef struct {
  uint32_t sig_kind;           /* carve_sig_kind of master and disk sectors; 0 = djb2-64 */
  float max_load;              /* load factor ceiling of the probed table in (0, 0.9]; 0 = 0.5
                                  (bucketed: keys per slot; linear: distinct signatures per slot;
                                  sorted: unused) */
  uint32_t bloom_bits_per_key; /* prefilter in front of the table: 0 = automatic (at least 4 bits per
                                  distinct signature, then as many as a 4 MiB filter and 16 bits allow;
                                  32 bits for a fragment index),
                                  CARVE_BLOOM_OFF = none, else 4..64 bits per signature */
  uint32_t layout;             /* carve_index_layout; 0 = bucketed */
  uint32_t reserved[4];        /* must be zero */
} carve_index_params;

#define CARVE_BLOOM_OFF 0xFFFFFFFFu

typedef struct {
  uint64_t disk_sector;    /* flagged disk sector id */
  uint32_t file_id;        /* master file index */
  uint32_t sector_in_file; /* sector index inside that file */
} carve_match;             /* 16 bytes */

typedef struct {
  uint64_t disk_sector;    /* flagged sector id within its image */
  uint32_t file_id;
  uint32_t sector_in_file;
  uint32_t image;          /* index of the image in the batch */
  uint32_t reserved;       /* 0 */
} carve_batch_match;       /* 24 bytes */

typedef struct {
  const void* image;       /* device, 16-B aligned (may be NULL when n_bytes < 512) */
  uint64_t n_bytes;        /* trailing n_bytes % 512 bytes are ignored */
  uint32_t tau0;           /* cluster position of the image's first sector, 0..7 */
  uint32_t tau_mode;       /* carve_tau_mode */
} carve_image_desc;        /* 24 bytes */

typedef struct {
  uint32_t blocks_per_cu;   /* work-groups of the persistent scan grid per compute unit; 0 = as many as fit */
  uint32_t tiles_per_chunk; /* consecutive 64-sector tiles a wave takes before striding (the split walk also
                               hands out the last eighth of each position's tiles in runs of this length); 0 = 1 */
  uint32_t split;           /* carve_split_mode: how scans of one image under the per-cluster rule walk it */
  uint32_t reserved;        /* must be zero */
} carve_scan_config;

/* The per-cluster rule (Section 3.1) lets a scan of one image be split by
 * cluster position: position p's sectors only need S_p, so the chip's 8 XCDs
 * each scan one position and keep one eighth of the prefilter in their L2. */
typedef enum {
  CARVE_SPLIT_AUTO = 0,     /* split when the prefilter is 4 MiB or more (too large for one XCD's L2) */
  CARVE_SPLIT_OFF = 1,      /* always scan contiguously */
  CARVE_SPLIT_ON = 2        /* always split (when the index has a prefilter) */
} carve_split_mode;

typedef struct {
  uint64_t n_master_sectors;
  uint64_t n_unique_signatures;  /* distinct signatures (any position) */
  uint64_t n_buckets;            /* 16-slot buckets of the hash table */
  uint64_t n_overflow_keys;      /* keys stored outside their home bucket */
  uint64_t device_bytes;         /* device memory owned by the index */
  uint64_t bloom_bytes;          /* size of the prefilter, 0 if none */
} carve_index_stats;

/*
 * build_master_index -- build the resident index of the master sectors
 * (Section 3.1, the tables S_tau and their linear-probing insertion, Eq. (3)).
 *   master_sectors      device, 16-B aligned, file_sector_offsets[n_files]
 *                       packed 512-byte sectors, file after file. BORROWED:
 *                       confirm_matches reads it, so it must stay valid and
 *                       unchanged until free_index.
 *   file_sector_offsets host, n_files+1 ascending values, [0] == 0; file f
 *                       owns sectors [off[f], off[f+1]) and its sector k sits
 *                       at cluster position k mod 8. A file's trailing
 *                       partial sector is not part of this array.
 *   params              host or NULL for defaults.
 *   stream              all work is enqueued on it; the call returns after
 *                       the build completes (it synchronizes the stream).
 *   out                 receives the new index (owned; release with free_index).
 * Errors: EINVAL (null out, misaligned or null masters with sectors > 0,
 * offsets not ascending or not starting at 0, bad params), EUNSUPPORTED
 * (2^32-1 or more master sectors, unknown sig_kind), ENOMEM, EDEVICE.
 */
int build_master_index(const void* master_sectors, const uint64_t* file_sector_offsets, uint32_t n_files,
                       const carve_index_params* params, void* stream, carve_index** out);

/*
 * scan_image -- signature, cluster position, index probe and flag compaction
 * of every whole sector of a device-resident image (Section 3.2 and the
 * filter of Section 3.1). Asynchronous: enqueued on `stream`.
 *   idx        index from build_master_index (not modified; several scans may
 *              use one index concurrently on different streams).
 *   image      device, 16-B aligned, n_bytes bytes. BORROWED until the scan is
 *              freed or reused. The trailing n_bytes % 512 bytes are ignored.
 *   tau0       cluster position of the image's first sector (0..7).
 *   tau_mode   carve_tau_mode.
 *   io         in: NULL to create a scan object, or a scan object to reuse
 *              (its previous results are discarded; it must not be in use on
 *              another stream). out: the scan object (release with free_scan).
 * Errors: EINVAL (null idx/io, null or misaligned image with n_bytes >= 512,
 * an image in host memory, tau0 > 7, bad tau_mode), ENOMEM, EDEVICE.
 */
int scan_image(const carve_index* idx, const void* image, uint64_t n_bytes, uint32_t tau0, uint32_t tau_mode,
               void* stream, carve_scan** io);

/*
 * flagged_sectors -- ascending ids of the flagged sectors of the last scan
 * (the match buffer of Section 3.2). Synchronizes the scan's stream.
 *   out    host or device, room for `cap` ids (may be NULL when cap == 0).
 *   n_out  host; receives the number of flagged sectors.
 * Returns ETRUNC (after copying the first cap ids) when the count exceeds cap.
 */
int flagged_sectors(carve_scan* sc, uint64_t* out, uint64_t cap, uint64_t* n_out);

/*
 * confirm_matches -- byte-for-byte confirmation of the flagged sectors of the
 * last scan (Section 3.1): every (flagged disk sector, master sector) pair
 * with equal signatures, a compatible cluster position and equal 512 bytes,
 * ordered by (disk_sector, file_id, sector_in_file), each pair once.
 * Runs on the scan's stream and synchronizes it.
 *   out    host or device, room for `cap` records (may be NULL when cap == 0).
 *   n_out  host; receives the number of confirmed pairs.
 * Returns ETRUNC (after copying the first cap records) when it exceeds cap.
 */
int confirm_matches(const carve_index* idx, carve_scan* sc, carve_match* out, uint64_t cap, uint64_t* n_out);

/*
 * confirm_enqueue -- enqueue the confirmation of the last scan on its stream
 * without waiting (the flagged count stays on the device); a later
 * confirm_matches then only copies the records out. Lets the whole hot path be
 * enqueued, or captured in a HIP graph, ahead of any readback. Calling
 * confirm_matches without it enqueues the work itself.
 * Graphs: a scan replayed from a captured graph runs no host code, so the
 * scan marks on the device that its confirmation is still to be done, and
 * confirm_matches checks that mark (one 8-byte readback) before reusing a
 * confirmation enqueued earlier: after replaying a graph that holds only the
 * scan, confirm_matches confirms the replayed scan; a graph that holds scan
 * and confirm_enqueue leaves only the copy to it.
 */
int confirm_enqueue(const carve_index* idx, carve_scan* sc);

/*
 * confirm_enqueue_to -- confirm_enqueue with the records written straight into
 * the caller's device memory (Section 3.1 confirmation; the host reads the
 * results once, Section 3.2): no copy afterwards. Asynchronous on the scan's
 * stream, nothing is read back, so a whole step (scan_image,
 * confirm_enqueue_to, flagged_sectors_enqueue, then scan_counts) waits once.
 *   out    device, room for cap records (may be NULL when cap == 0); receives
 *          the first min(matches, cap) records in confirm_matches' order.
 *          BORROWED until the stream has run the confirmation.
 * A later confirm_matches with the same out and cap reads the count only.
 * Errors: EINVAL (null idx/sc, a batch object, another index, null out with
 * cap > 0, out not device memory), ENOMEM, EDEVICE.
 */
int confirm_enqueue_to(const carve_index* idx, carve_scan* sc, carve_match* out, uint64_t cap);

/*
 * flagged_sectors_enqueue -- flagged_sectors into the caller's device memory
 * without waiting: enqueues the copy of the first min(count, cap) ids on the
 * scan's stream (Section 3.2's match buffer). The count comes from
 * scan_counts (or flagged_sectors) afterwards.
 *   out    device, room for cap ids (may be NULL when cap == 0).
 * Errors: EINVAL (null sc, a batch object, null out with cap > 0, out not
 * device memory), EDEVICE.
 */
int flagged_sectors_enqueue(carve_scan* sc, uint64_t* out, uint64_t cap);

/*
 * scan_counts -- synchronizes the scan's stream and reads its counts in one
 * readback: the flagged units of the latest scan (a batch: of all its images)
 * and the records of a confirmation that ran after it, or
 * CARVE_NOT_CONFIRMED when none did.
 * Errors: EINVAL (null argument), EDEVICE.
 */
int scan_counts(carve_scan* sc, uint64_t* n_flagged, uint64_t* n_confirmed);

/*
 * scan_wait_kernel -- makes `stream` (a hipStream_t, or NULL for the null
 * stream) wait until the latest scan kernel of `sc` has finished, not the
 * compaction and confirmation enqueued after it on the scan's stream: work
 * enqueued on `stream` afterwards (another scan object's scan, say) may then
 * run beside them. Nothing to wait for before the first scan. An ordering
 * point only: no results are handed over (the scan's outputs are read after
 * its compaction, on its own stream), so the wait carries no system-scope
 * cache fence. For keeping several steps in flight on several streams
 * (Section 3.2's pipeline of scans, with the host never waiting between
 * them).
 * Errors: EINVAL (null sc), EDEVICE.
 */
int scan_wait_kernel(carve_scan* sc, void* stream);
#define CARVE_NOT_CONFIRMED UINT64_MAX

/*
 * sector_signatures -- djb2-64 signature (Eq. (1), Section 4) of each of
 * n_sectors packed sectors. sectors: device, 16-B aligned; sigs: device,
 * n_sectors values. Asynchronous on `stream`.
 */
int sector_signatures(const void* sectors, uint64_t n_sectors, uint64_t* sigs, void* stream);

/* sector_signatures_kind -- sector_signatures for a carve_sig_kind (djb2-64,
 * Eq. (1); or CRC-64, Section 2.1). EINVAL for an unknown kind. */
int sector_signatures_kind(uint32_t sig_kind, const void* sectors, uint64_t n_sectors, uint64_t* sigs,
                           void* stream);

/* ---------------------------------------------------------------- fragments
 * Section 5 scans every 64-byte fragment of a disk aligned on a 32-bit
 * boundary, to find small files (logos, images) embedded in others. Master
 * fragment k of a file is its bytes [64k, 64k + 64); window j of an image is
 * its bytes [4j, 4j + 64), for every j with 4j + 64 <= n_bytes. A window is
 * flagged when its djb2-64 signature (Eq. (1) over the 64 bytes) is that of a
 * master fragment, at any position (no cluster rule); confirmation compares
 * the 64 bytes. The scan object is the one of scan_image: flagged_sectors
 * returns window ids j (byte offset 4j), confirm_matches / confirm_enqueue
 * records (disk_sector = j, file_id, sector_in_file = fragment index).
 */

/* build_fragment_index -- as build_master_index, over packed 64-byte master
 * fragments: master_fragments: device, 16-B aligned, file_fragment_offsets[n_files]
 * fragments of 64 B; file_fragment_offsets: host CSR (n_files + 1 entries,
 * [0] = 0) of each file's fragment range. params as build_master_index;
 * EUNSUPPORTED unless sig_kind is djb2-64 and layout is bucketed. The index
 * serves scan_fragments only (scan_image, scan_batch, autotune_scan and
 * server_create reject it with EINVAL). index_stats counts fragments as
 * master sectors. */
int build_fragment_index(const void* master_fragments, const uint64_t* file_fragment_offsets, uint32_t n_files,
                         const carve_index_params* params, void* stream, carve_index** out);

/* scan_fragments -- flag every window of a device-resident image (16-B
 * aligned; any n_bytes; fewer than 64 bytes gives no window). Asynchronous on
 * `stream`; *io as scan_image (reused when non-null). EINVAL for a sector
 * index, a null, misaligned or host-memory image, or a batch object. The scan
 * object keeps about 15 bytes of device workspace per window; its
 * confirmation first reserves room for an eighth of the windows and
 * confirm_matches redoes it, with room for all, when more were flagged. */
int scan_fragments(const carve_index* idx, const void* image, uint64_t n_bytes, void* stream, carve_scan** io);

/* ---------------------------------------------------------------- host ingest
 * Section 3.1 (Fig. 7): images in host memory, streamed to the GPU by chunks
 * through a pair of device buffers while the other chunk is scanned; a
 * pageable image goes through a pair of pinned host buffers filled by CPU
 * threads, a pinned one (hipHostMalloc) is transferred directly. Results are
 * those of scan_image / confirm_matches on the whole image (ids relative to
 * its first sector). One thread drives an ingest object.
 */
typedef struct carve_ingest carve_ingest;

typedef struct {
  uint64_t chunk_bytes;        /* bytes per transfer, a multiple of 4096 (chunks keep the image's
                                  cluster positions); 0 = 256 MiB. Device and pinned memory: 2 each */
  uint32_t confirm;            /* non-zero: confirm the flagged sectors */
  uint32_t copy_threads;       /* CPU threads staging a pageable image; 0 = 8, at most 64 */
  uint32_t reserved[4];        /* must be zero */
} carve_ingest_params;

typedef struct {
  uint64_t bytes;              /* bytes scanned by the last ingest_scan (whole sectors) */
  uint64_t chunks;
  double seconds;              /* its wall time, transfers included */
  uint32_t pinned_source;      /* 1: the image was pinned and transferred directly */
  uint32_t reserved;
} carve_ingest_stats;

/* ingest_create -- idx (a sector index) must outlive the object. EINVAL for a
 * bad chunk size or a fragment index, ENOMEM when buffers fail. */
int ingest_create(const carve_index* idx, const carve_ingest_params* params, carve_ingest** out);

/* ingest_scan -- scan host_image (host pointer, n_bytes; the trailing partial
 * sector is ignored) with tau0 / tau_mode as scan_image; returns when every
 * chunk is scanned (and confirmed) and its results collected. */
int ingest_scan(carve_ingest* in, const void* host_image, uint64_t n_bytes, uint32_t tau0, uint32_t tau_mode);

/* ingest_flagged_sectors / ingest_matches -- the last ingest_scan's ascending
 * flagged sector ids / ordered records (host buffers; ETRUNC + full count when
 * short; records only with confirm set). */
int ingest_flagged_sectors(const carve_ingest* in, uint64_t* out, uint64_t cap, uint64_t* n_out);
int ingest_matches(const carve_ingest* in, carve_match* out, uint64_t cap, uint64_t* n_out);
int ingest_stats(const carve_ingest* in, carve_ingest_stats* out);
void ingest_free(carve_ingest* in);   /* NULL is a no-op; waits for transfers and scans in flight */

/*
 * scan_image_noalloc -- scan_image followed by flagged_sectors into device
 * memory, for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc). It allocates nothing:
 * its work buffers are one fixed device array of the library, 32 MiB + 34 KiB,
 * that every GPU running the library holds until the process ends. It records
 * no confirmation data (there is no scan object for confirm_matches).
 *   idx, image, n_bytes, tau0, tau_mode, stream   as scan_image; at most 2^27
 *          sectors (64 GiB), EINVAL beyond.
 *   ids    device, room for cap ids (may be NULL when cap == 0): receives the
 *          first min(count, cap) flagged sector ids, ascending.
 *   count  device, one uint64_t: receives the number of flagged sectors (the
 *          full count, also when it exceeds cap).
 * Asynchronous on `stream`: nothing is read back. Every call on one GPU uses
 * that GPU's one array, so calls that overlap on a GPU (on any streams) race:
 * the caller orders them (e.g. one stream).
 * Errors: EINVAL (as scan_image; also ids or count not 8-byte aligned or not
 * device memory, a fragment index, too many sectors), EDEVICE.
 */
int scan_image_noalloc(const carve_index* idx, const void* image, uint64_t n_bytes, uint32_t tau0, uint32_t tau_mode,
                       void* stream, uint64_t* ids, uint64_t cap, uint64_t* count);

/*
 * read_ceiling_probe -- the streaming-read rate the scan kernels are measured
 * against: one kernel reads the whole sectors of a device image once with a
 * scan kernel's access pattern (64-sector tiles, 16 B per lane with
 * non-temporal loads, two phases of a tile in flight, a resident grid) and no
 * other work. Not a step of the method; a measurement of the chip.
 *   pattern        0: contiguous tiles (as the contiguous scan); 1: split by
 *                  cluster position (as the position-split scan).
 *   blocks_per_cu  resident work-groups per CU; 0 = as many as fit.
 *   ms             host; receives the kernel's duration (HIP events).
 * Synchronizes `stream`. EINVAL for fewer than 512 whole sectors, a
 * misaligned or non-device image, a bad pattern.
 */
int read_ceiling_probe(const void* image, uint64_t n_bytes, uint32_t pattern, uint32_t blocks_per_cu, void* stream,
                       float* ms);

/* index_stats -- sizes of a built index (host struct). */
int index_stats(const carve_index* idx, carve_index_stats* out);

/*
 * index_set_scan_config / index_get_scan_config -- launch shape of the scan
 * kernel for scans with this index (results never depend on it). Setting it
 * while scans are being enqueued on other threads is a race.
 */
int index_set_scan_config(carve_index* idx, const carve_scan_config* cfg);
int index_get_scan_config(const carve_index* idx, carve_scan_config* cfg);

/*
 * autotune_scan -- time the scan kernel for each candidate launch shape on a
 * sample image (device, 16-B aligned, n_bytes >= 512) and keep the fastest
 * for the index; *best (host, may be NULL) receives it. Synchronizes stream.
 */
int autotune_scan(carve_index* idx, const void* sample_image, uint64_t n_bytes, void* stream, carve_scan_config* best);

/*
 * autotune_index -- build_master_index with the index layout, the prefilter
 * size and the scan's launch shape picked by timing them on a sample image
 * (the occupancy and layout study of Section 4, the probe of Eq. (3)). Every
 * choice gives the same results; only the time differs.
 *   Stage 1 builds each candidate (layout x prefilter bits per signature) from
 *   `base` and times its scan of the sample at one launch shape, contiguous
 *   and position-split; stage 2 sweeps the fastest candidate's launch shapes
 *   (as autotune_scan). The pick is cached for the process under the device's
 *   architecture, the signature kind, the master count's power-of-two class,
 *   max_load and the space: a later call with the same key builds the cached
 *   pick without timing.
 *   master_sectors, file_sector_offsets, n_files, base   as build_master_index
 *                  (base: host or NULL; its layout and bloom_bits_per_key are
 *                  replaced by each candidate's).
 *   space          host or NULL (every layout; the automatic prefilter and 8,
 *                  16 and 32 bits per signature).
 *   sample_image   device, 16-B aligned, at least one sector: an image like
 *                  the ones to be scanned (not necessarily one of them).
 *   out            receives the picked index with the picked launch shape.
 *   result         host or NULL: what was picked.
 * Synchronizes `stream`. Errors as build_master_index and autotune_scan.
 */
#define CARVE_TUNE_NO_CACHE 1u    /* time the candidates even when the key is cached (and cache the new pick) */
#define CARVE_TUNE_CONTIGUOUS 2u  /* the index will serve batches (scan_batch, the server): time the batch
                                     kernel, over the sample cut into 16 images of uneven sizes */
typedef struct {
  uint32_t layouts;        /* bit l: try carve_index_layout l; 0 = all three */
  uint32_t n_bloom;        /* entries of bloom_bits (at most 8); 0 = {0 (automatic), 8, 16, 32} */
  uint32_t bloom_bits[8];  /* bloom_bits_per_key candidates (0 = automatic, CARVE_BLOOM_OFF = none, 4..64) */
  uint32_t flags;          /* CARVE_TUNE_* */
  uint32_t reserved[2];    /* must be zero */
} carve_tune_space;

typedef struct {
  carve_index_params params;  /* the picked build parameters */
  carve_scan_config config;   /* the picked launch shape (already set on the index) */
  float kernel_ms;            /* mean scan-kernel time of the pick on the sample (cached: when it was timed) */
  uint32_t candidates;        /* indexes built and timed (0 when taken from the cache) */
  uint32_t from_cache;        /* 1: the pick came from the cache */
  uint32_t reserved;
} carve_tune_result;

int autotune_index(const void* master_sectors, const uint64_t* file_sector_offsets, uint32_t n_files,
                   const carve_index_params* base, const carve_tune_space* space, const void* sample_image,
                   uint64_t n_bytes, void* stream, carve_index** out, carve_tune_result* result);

/*
 * scan_batch -- scan_image over n_images images at once: one persistent
 * launch over all their sectors, flags compacted per image (the paper scans
 * several disks at once, Section 3). Asynchronous on `stream`.
 *   images   host array of n_images descriptors (images BORROWED as in scan_image).
 *   io       in: NULL to create a batch object, or one to reuse; out: the batch.
 * When every descriptor equals the previous call's, nothing but kernels is
 * enqueued, so a reused call can be captured in a HIP graph and replayed.
 * Errors: EINVAL (null idx/io/images with n_images > 0, bad descriptor --
 * which names the image --, new descriptors during stream capture), ENOMEM, EDEVICE.
 */
int scan_batch(const carve_index* idx, const carve_image_desc* images, uint32_t n_images, void* stream,
               carve_batch** io);

/* batch_flag_counts -- flagged sectors per image (host array of n_images). Synchronizes. */
int batch_flag_counts(carve_batch* b, uint64_t* counts, uint32_t n_images);

/* batch_flagged_sectors -- flagged_sectors for image `image` of the batch, or,
 * with image == CARVE_ALL_IMAGES, the ids of every image one after the other
 * in image order (split them with batch_flag_counts). Synchronizes. */
int batch_flagged_sectors(carve_batch* b, uint32_t image, uint64_t* out, uint64_t cap, uint64_t* n_out);
#define CARVE_ALL_IMAGES 0xFFFFFFFFu

/*
 * batch_confirm_matches -- confirm_matches for every image of the batch,
 * ordered by (image, disk_sector, file_id, sector_in_file). Synchronizes.
 */
int batch_confirm_matches(const carve_index* idx, carve_batch* b, carve_batch_match* out, uint64_t cap,
                          uint64_t* n_out);

/* batch_confirm_enqueue -- confirm_enqueue for a batch (the same rule for
 * graphs holding only scan_batch). */
int batch_confirm_enqueue(const carve_index* idx, carve_batch* b);

/* scan_set_timing -- when enable != 0, later scans through this object
 * (scan_image, scan_fragments, scan_batch) bracket the signature/probe kernel
 * with HIP events on the scan's stream; switching it on when it was off starts
 * a new series for scan_kernel_ms_recent. EDEVICE if the events cannot be
 * created. */
int scan_set_timing(carve_scan* sc, int enable);

/* scan_kernel_ms -- duration of the signature/probe kernel of the last timed
 * scan, in milliseconds (synchronizes on its end event). EINVAL if the last
 * scan was not timed. */
int scan_kernel_ms(carve_scan* sc, float* ms);

/* scan_kernel_ms_recent -- durations of the signature/probe kernels of the
 * last min(n, timed launches, 256) timed scans since timing was switched on, oldest
 * first, into ms (host, n floats); *n_out receives how many. Synchronizes once,
 * on the end event of the latest, so a timed loop can read them all after it
 * ends. A scan replayed from a captured graph re-records the events of the
 * launch that was captured. */
int scan_kernel_ms_recent(carve_scan* sc, float* ms, uint32_t n, uint32_t* n_out);

/* ---------------------------------------------------------------- serving
 * A request loop over one resident index: scan jobs (disk-image chunks or
 * flow buffers) are queued, admitted in arrival order while the image bytes
 * admitted and not yet completed stay within a budget, and launched as one
 * batch per free stream lane, so jobs that arrive while others run join the
 * next batch (continuous batching) and batches on different lanes overlap on
 * the device. Each job is scanned and, optionally, confirmed exactly as
 * scan_image + confirm_matches would do it alone. Not thread-safe: one
 * thread drives a server.
 */
typedef struct carve_server carve_server;

typedef struct {
  uint32_t n_streams;          /* stream lanes (concurrent batches); 0 = 2. A lane whose batch
                                  starts while another lane's runs scans on half of the CUs' slots */
  uint32_t max_jobs_per_batch; /* 0 = 4096; at most 65536 */
  uint64_t budget_bytes;       /* image bytes admitted and not completed; 0 = 32 GiB */
  uint32_t confirm;            /* non-zero: confirm each job's flagged sectors */
  uint32_t reserved[3];        /* must be zero */
} carve_server_params;

typedef struct {
  uint64_t job_id;
  uint64_t n_flagged;
  uint64_t n_confirmed;        /* 0 when the server does not confirm */
  int32_t status;              /* CARVE_OK or the error of its batch */
  uint32_t reserved;
} carve_job_done;

typedef struct {
  uint64_t queued_jobs, running_jobs, done_jobs;   /* done: completed and not yet released */
  uint64_t in_flight_bytes;                        /* admitted, not completed */
  uint64_t batches_launched, jobs_completed;
  double host_launch_s;                            /* host time spent admitting and launching */
  double host_retire_s;                            /* host time spent collecting results */
} carve_server_stats;

/* server_create -- idx must outlive the server. params: host or NULL.
 * Device memory: each lane's workspace is sized up front for batches of
 * budget_bytes / n_streams (about 40 bytes per 512-byte sector: ids, match
 * slots, confirmation scratch, records), so serving allocates nothing unless a
 * batch exceeds that share; pinned host memory holds one such batch's ids and
 * records per lane; the first host-memory job of a lane allocates its arena
 * (the lane's share of the budget). EINVAL for n_streams > 64 or
 * max_jobs_per_batch > 65536. */
int server_create(const carve_index* idx, const carve_server_params* params, carve_server** out);

/* server_submit -- queue a job (host descriptor, image BORROWED until the job is
 * released). The image may be in device memory, or in host memory (sectors
 * arriving from disks through host memory, Section 3.1): a host job is copied
 * into its lane's device arena at launch, asynchronously when the memory is
 * pinned (hipHostMalloc), blocking the polling thread while it copies when it
 * is pageable. EINVAL for a bad descriptor, EUNSUPPORTED when the job alone
 * exceeds the budget. *job_id receives its id. Does not launch anything. */
int server_submit(carve_server* s, const carve_image_desc* job, uint64_t* job_id);

/* server_submit_many -- server_submit of jobs[0..n) in order, ids into
 * job_ids[0..n) (host arrays). All or nothing: when a descriptor is rejected no
 * job is queued and the message names the first bad one. For clients that
 * hand over many jobs at once without a call per job. */
int server_submit_many(carve_server* s, const carve_image_desc* jobs, uint32_t n, uint64_t* job_ids);

/* server_poll -- non-blocking progress: retire finished batches, admit queued
 * jobs into free lanes and launch them. Completed jobs are reported once,
 * in `done` (host, cap entries); *n_done receives how many were written (the
 * rest are reported by later calls). A batch that fails to launch or to
 * retire reports each of its jobs with the error as its `status` (the call
 * returns CARVE_OK); the call's own error is EINVAL for a bad argument and
 * EDEVICE when a lane's completion cannot be queried (its jobs stay running). */
int server_poll(carve_server* s, carve_job_done* done, uint32_t cap, uint32_t* n_done);

/* server_job_flags / server_job_matches -- results of a completed job
 * (host buffers; ETRUNC + full count when short, EINVAL if not completed, the
 * job's own error status if it failed: a failed job has no results). */
int server_job_flags(carve_server* s, uint64_t job_id, uint64_t* out, uint64_t cap, uint64_t* n_out);
int server_job_matches(carve_server* s, uint64_t job_id, carve_match* out, uint64_t cap, uint64_t* n_out);

/* server_release -- forget a completed job's results. */
int server_release(carve_server* s, uint64_t job_id);

/* server_release_many -- server_release of job_ids[0..n) (host array) in
 * order; stops at the first id that is not a reported job (EINVAL), the ids
 * before it released. */
int server_release_many(carve_server* s, const uint64_t* job_ids, uint32_t n);

/* server_fail_next_launches -- for tests of the failure path: the next n
 * batch launches fail with CARVE_EDEVICE after all of their work (host-job
 * copies, scan, confirmation, stage-out) has been enqueued. The server then
 * does what it does for any launch error: it waits for the lane's stream,
 * reports each of the batch's jobs with that status (server_poll) and frees
 * their budget. Jobs that fail this way have no results; submit them again.
 * EINVAL for a NULL server. */
int server_fail_next_launches(carve_server* s, uint32_t n);

int server_stats(const carve_server* s, carve_server_stats* out);
void server_free(carve_server* s);  /* NULL is a no-op; waits for running batches */

void free_index(carve_index* idx);  /* NULL is a no-op; the caller ensures no scan is running */
void free_scan(carve_scan* sc);     /* NULL is a no-op; waits for the scan's stream */
void free_batch(carve_batch* b);    /* NULL is a no-op; waits for the batch's stream */
const char* carve_last_error(void); /* message of this thread's last failure, "" if none */

#ifdef __cplusplus
}
#endif

#endif /* CARVE_H */
