/*
 * carve_oracle.c -- CPU oracle for hash-based sector carving.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header, table or constant with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (Collange, Dandass, Daumas, Defour, "Using Graphics
 * Processors for Parallelizing Hash-based Data Carving"):
 *   - the signature of a 512-byte sector is djb2 (Eq. (1), Section 2.2) with a
 *     64-bit accumulator (Section 4): h = 5381, then h = h*33 + s for every
 *     byte s (unsigned, in address order), modulo 2^64;
 *   - or, as the other signature the paper times (Section 2.1, Figs. 10-11),
 *     a 64-bit CRC. The paper does not give its parameters; the reading taken
 *     is CRC-64/GO-ISO: generator x^64 + x^4 + x^3 + x + 1, bytes fed least
 *     significant bit first (reflected in and out), register preset to all
 *     ones and the result complemented. It is computed bit by bit below, as
 *     polynomial division, with no table;
 *   - master entries: sector k of master file f sits at cluster position
 *     tau = k mod 8 (Section 3.1, the per-position tables S_tau, with the
 *     8-sector cluster of Section 2);
 *   - a disk sector j is flagged when some master entry has the same
 *     signature and a compatible position: tau == (j + tau0) mod 8 for the
 *     per-cluster rule of Section 3.1, or any position when the caller asks
 *     for it (buffers with no cluster alignment);
 *   - confirmation (Section 3.1) keeps the (disk sector, master) pairs of a
 *     flagged sector whose 512 bytes are equal;
 *   - fragments (Section 5): the unit can instead be a 64-byte fragment. Master
 *     fragment k of a file is its bytes [64k, 64k + 64); the image is read as
 *     every 64-byte window that starts on a 4-byte boundary (window j covers
 *     bytes [4j, 4j + 64)), matched at any position, confirmed by comparing the
 *     64 bytes.
 * The membership test here is a sorted array searched by bisection, not a
 * hash table: the result is a set, and the oracle only has to be plainly
 * correct. A brute-force all-pairs byte comparison is provided as well.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SECTOR_BYTES 512u
#define CLUSTER_SECTORS 8u

typedef struct {
  uint64_t sig;
  uint64_t master;   /* index of the sector in the packed master array */
  uint32_t file;
  uint32_t k;        /* sector index inside its file */
} oracle_entry;

typedef struct {
  uint64_t disk_sector;
  uint32_t file_id;
  uint32_t sector_in_file;
} oracle_match;

typedef struct {
  oracle_entry* e;
  uint64_t n;
  const uint8_t* masters;
  int sig_kind;      /* ORACLE_SIG_DJB2 or ORACLE_SIG_CRC64_GO_ISO */
  uint32_t unit;     /* bytes per master unit: a sector (512) or a fragment (64) */
} oracle_index;

#define FRAGMENT_BYTES 64u
#define WINDOW_STRIDE 4u

enum { ORACLE_SIG_DJB2 = 0, ORACLE_SIG_CRC64_GO_ISO = 1 };

/* ---------------------------------------------------------------- Eq. (1) */
uint64_t oracle_djb2(const uint8_t* s, uint64_t len) {
  uint64_t h = 5381u;
  for (uint64_t i = 0; i < len; i++) h = h * 33u + (uint64_t)s[i];
  return h;
}

/* ------------------------------------------------------ CRC-64 (Sec. 2.1) */
/* Generator polynomial without its x^64 term, most significant bit = x^63. */
#define CRC64_GO_ISO_POLY 0x000000000000001Bull

static uint64_t reverse64(uint64_t x) {
  uint64_t r = 0;
  for (int i = 0; i < 64; i++) r |= ((x >> i) & 1u) << (63 - i);
  return r;
}

/* Reflected CRC: each input byte enters least significant bit first, so the
 * register shifts right, its bit 0 is the coefficient that leaves next, and
 * the generator is applied in bit-reversed form (bit 63 = x^0, bit 0 = x^63). */
uint64_t oracle_crc64(const uint8_t* s, uint64_t len) {
  const uint64_t poly_reflected = reverse64(CRC64_GO_ISO_POLY);
  uint64_t crc = ~0ull;                       /* preset to all ones */
  for (uint64_t i = 0; i < len; i++) {
    crc ^= (uint64_t)s[i];
    for (int b = 0; b < 8; b++) crc = (crc & 1u) ? (crc >> 1) ^ poly_reflected : crc >> 1;
  }
  return ~crc;                                /* complemented result */
}

static uint64_t signature_n(int kind, const uint8_t* s, uint64_t len) {
  return kind == ORACLE_SIG_CRC64_GO_ISO ? oracle_crc64(s, len) : oracle_djb2(s, len);
}

static uint64_t signature(int kind, const uint8_t* s) {
  return kind == ORACLE_SIG_CRC64_GO_ISO ? oracle_crc64(s, SECTOR_BYTES) : oracle_djb2(s, SECTOR_BYTES);
}

/* --------------------------------------------------------------- threads */
typedef struct {
  void (*fn)(void* ctx, uint64_t lo, uint64_t hi, int t);
  void* ctx;
  uint64_t lo, hi;
  int t;
} oracle_job;

static void* oracle_run_job(void* p) {
  oracle_job* j = (oracle_job*)p;
  j->fn(j->ctx, j->lo, j->hi, j->t);
  return NULL;
}

static void parallel_for(uint64_t n, int threads, void (*fn)(void*, uint64_t, uint64_t, int), void* ctx) {
  if (threads < 1) threads = 1;
  if ((uint64_t)threads > n) threads = n ? (int)n : 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * threads);
  oracle_job* jobs = (oracle_job*)malloc(sizeof(oracle_job) * threads);
  for (int t = 0; t < threads; t++) {
    jobs[t].fn = fn;
    jobs[t].ctx = ctx;
    jobs[t].lo = n * (uint64_t)t / threads;
    jobs[t].hi = n * (uint64_t)(t + 1) / threads;
    jobs[t].t = t;
  }
  for (int t = 1; t < threads; t++) pthread_create(&th[t], NULL, oracle_run_job, &jobs[t]);
  oracle_run_job(&jobs[0]);
  for (int t = 1; t < threads; t++) pthread_join(th[t], NULL);
  free(jobs);
  free(th);
}

/* ------------------------------------------------------ sector signatures */
typedef struct {
  const uint8_t* data;
  uint64_t* out;
  int kind;
} sig_ctx;

static void sig_range(void* p, uint64_t lo, uint64_t hi, int t) {
  (void)t;
  sig_ctx* c = (sig_ctx*)p;
  for (uint64_t i = lo; i < hi; i++) c->out[i] = signature(c->kind, c->data + i * SECTOR_BYTES);
}

void oracle_sector_signatures_kind(const uint8_t* data, uint64_t n_sectors, uint64_t* out, int threads,
                                   int kind) {
  sig_ctx c = {data, out, kind};
  parallel_for(n_sectors, threads, sig_range, &c);
}

void oracle_sector_signatures(const uint8_t* data, uint64_t n_sectors, uint64_t* out, int threads) {
  oracle_sector_signatures_kind(data, n_sectors, out, threads, ORACLE_SIG_DJB2);
}

/* ------------------------------------------------------------ the index */
static int entry_cmp(const void* a, const void* b) {
  const oracle_entry* x = (const oracle_entry*)a;
  const oracle_entry* y = (const oracle_entry*)b;
  if (x->sig != y->sig) return x->sig < y->sig ? -1 : 1;
  if (x->master != y->master) return x->master < y->master ? -1 : 1;
  return 0;
}

typedef struct {
  const uint8_t* masters;
  const uint64_t* file_offsets;
  uint32_t n_files;
  oracle_entry* e;
  int kind;
  uint32_t unit;
} build_ctx;

static void build_range(void* p, uint64_t lo, uint64_t hi, int t) {
  (void)t;
  build_ctx* c = (build_ctx*)p;
  uint32_t f = 0;
  for (uint64_t m = lo; m < hi; m++) {
    while (f + 1 < c->n_files && c->file_offsets[f + 1] <= m) f++;
    c->e[m].sig = signature_n(c->kind, c->masters + m * c->unit, c->unit);
    c->e[m].master = m;
    c->e[m].file = f;
    c->e[m].k = (uint32_t)(m - c->file_offsets[f]);
  }
}

/* masters: n = file_offsets[n_files] packed sectors; file f owns sectors
 * [file_offsets[f], file_offsets[f+1]). The masters buffer must outlive the index. */
static void* build_units(const uint8_t* masters, const uint64_t* file_offsets, uint32_t n_files, int threads,
                         int kind, uint32_t unit) {
  oracle_index* ix = (oracle_index*)calloc(1, sizeof(oracle_index));
  ix->n = n_files ? file_offsets[n_files] : 0;
  ix->masters = masters;
  ix->sig_kind = kind;
  ix->unit = unit;
  ix->e = (oracle_entry*)malloc(sizeof(oracle_entry) * (ix->n ? ix->n : 1));
  build_ctx c = {masters, file_offsets, n_files, ix->e, kind, unit};
  /* file lookup walks forward from 0 in each range: fine for tests */
  parallel_for(ix->n, threads, build_range, &c);
  qsort(ix->e, ix->n, sizeof(oracle_entry), entry_cmp);
  return ix;
}

void* oracle_build_kind(const uint8_t* masters, const uint64_t* file_offsets, uint32_t n_files, int threads,
                        int kind) {
  return build_units(masters, file_offsets, n_files, threads, kind, SECTOR_BYTES);
}

void* oracle_build(const uint8_t* masters, const uint64_t* file_offsets, uint32_t n_files, int threads) {
  return oracle_build_kind(masters, file_offsets, n_files, threads, ORACLE_SIG_DJB2);
}

/* masters: packed 64-byte fragments; file f owns fragments [file_offsets[f], file_offsets[f+1]). */
void* oracle_build_fragments(const uint8_t* fragments, const uint64_t* file_offsets, uint32_t n_files, int threads) {
  return build_units(fragments, file_offsets, n_files, threads, ORACLE_SIG_DJB2, FRAGMENT_BYTES);
}

void oracle_free(void* p) {
  oracle_index* ix = (oracle_index*)p;
  if (!ix) return;
  free(ix->e);
  free(ix);
}

uint64_t oracle_index_size(void* p) { return ((oracle_index*)p)->n; }

/* first entry with e.sig >= sig */
static uint64_t lower_bound(const oracle_index* ix, uint64_t sig) {
  uint64_t lo = 0, hi = ix->n;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (ix->e[mid].sig < sig) lo = mid + 1; else hi = mid;
  }
  return lo;
}

static int tau_ok(const oracle_entry* e, uint64_t j, uint32_t tau0, int any_tau) {
  return any_tau || (e->k % CLUSTER_SECTORS) == (uint32_t)((j + tau0) % CLUSTER_SECTORS);
}

static int is_flagged(const oracle_index* ix, uint64_t sig, uint64_t j, uint32_t tau0, int any_tau) {
  for (uint64_t p = lower_bound(ix, sig); p < ix->n && ix->e[p].sig == sig; p++)
    if (tau_ok(&ix->e[p], j, tau0, any_tau)) return 1;
  return 0;
}

/* ------------------------------------------------------------ flagging */
typedef struct {
  const oracle_index* ix;
  const uint8_t* image;
  const uint64_t* ids;     /* NULL: sector i of the image is sector i */
  uint32_t tau0;
  int any_tau;
  uint8_t* flag;           /* one byte per sector */
} flag_ctx;

static void flag_range(void* p, uint64_t lo, uint64_t hi, int t) {
  (void)t;
  flag_ctx* c = (flag_ctx*)p;
  for (uint64_t i = lo; i < hi; i++) {
    uint64_t j = c->ids ? c->ids[i] : i;
    uint64_t h = signature(c->ix->sig_kind, c->image + i * SECTOR_BYTES);
    c->flag[i] = (uint8_t)is_flagged(c->ix, h, j, c->tau0, c->any_tau);
  }
}

/* Flags of n sectors whose bytes are packed in `sectors`; ids[i] is the disk
 * sector number of the i-th one (for its cluster position), or NULL for 0..n-1. */
void oracle_flag_sectors(void* p, const uint8_t* sectors, const uint64_t* ids, uint64_t n,
                         uint32_t tau0, int any_tau, uint8_t* flag_out, int threads) {
  flag_ctx c = {(const oracle_index*)p, sectors, ids, tau0, any_tau, flag_out};
  parallel_for(n, threads, flag_range, &c);
}

/* Ascending ids of the flagged sectors of an image of n_bytes bytes (the
 * trailing partial sector is not scanned). Returns the count; writes at most cap. */
int64_t oracle_flag_image(void* p, const uint8_t* image, uint64_t n_bytes, uint32_t tau0, int any_tau,
                          uint64_t* out, uint64_t cap, int threads) {
  uint64_t n = n_bytes / SECTOR_BYTES;
  uint8_t* flag = (uint8_t*)malloc(n ? n : 1);
  oracle_flag_sectors(p, image, NULL, n, tau0, any_tau, flag, threads);
  uint64_t cnt = 0;
  for (uint64_t j = 0; j < n; j++)
    if (flag[j]) {
      if (cnt < cap) out[cnt] = j;
      cnt++;
    }
  free(flag);
  return (int64_t)cnt;
}

/* --------------------------------------------------------- confirmation */
/* For each flagged sector (ascending), every master entry with an equal
 * signature and a compatible position whose bytes are equal, in master order
 * (file, then sector in file). `sectors` holds the bytes of the flagged
 * sectors in the same order as `ids`. */
int64_t oracle_confirm(void* p, const uint8_t* sectors, const uint64_t* ids, uint64_t n,
                       uint32_t tau0, int any_tau, oracle_match* out, uint64_t cap) {
  const oracle_index* ix = (const oracle_index*)p;
  uint64_t cnt = 0;
  for (uint64_t i = 0; i < n; i++) {
    const uint8_t* s = sectors + i * SECTOR_BYTES;
    uint64_t h = signature(ix->sig_kind, s);
    for (uint64_t q = lower_bound(ix, h); q < ix->n && ix->e[q].sig == h; q++) {
      const oracle_entry* e = &ix->e[q];
      if (!tau_ok(e, ids[i], tau0, any_tau)) continue;
      if (memcmp(s, ix->masters + e->master * SECTOR_BYTES, SECTOR_BYTES) != 0) continue;
      if (cnt < cap) {
        out[cnt].disk_sector = ids[i];
        out[cnt].file_id = e->file;
        out[cnt].sector_in_file = e->k;
      }
      cnt++;
    }
  }
  return (int64_t)cnt;
}

/* ------------------------------------------------------------ brute force */
typedef struct {
  const uint8_t* image;
  const uint8_t* masters;
  const uint64_t* file_offsets;
  uint32_t n_files;
  uint32_t tau0;
  int any_tau;
  oracle_match** part;
  uint64_t* part_n;
  uint64_t* part_cap;
} brute_ctx;

static void brute_range(void* p, uint64_t lo, uint64_t hi, int t) {
  brute_ctx* c = (brute_ctx*)p;
  uint64_t n_m = c->n_files ? c->file_offsets[c->n_files] : 0;
  for (uint64_t j = lo; j < hi; j++) {
    const uint8_t* d = c->image + j * SECTOR_BYTES;
    uint32_t f = 0;
    for (uint64_t m = 0; m < n_m; m++) {
      while (f + 1 < c->n_files && c->file_offsets[f + 1] <= m) f++;
      uint32_t k = (uint32_t)(m - c->file_offsets[f]);
      if (!c->any_tau && k % CLUSTER_SECTORS != (uint32_t)((j + c->tau0) % CLUSTER_SECTORS)) continue;
      if (memcmp(d, c->masters + m * SECTOR_BYTES, SECTOR_BYTES) != 0) continue;
      if (c->part_n[t] == c->part_cap[t]) {
        c->part_cap[t] = c->part_cap[t] ? 2 * c->part_cap[t] : 256;
        c->part[t] = (oracle_match*)realloc(c->part[t], sizeof(oracle_match) * c->part_cap[t]);
      }
      oracle_match* o = &c->part[t][c->part_n[t]++];
      o->disk_sector = j;
      o->file_id = f;
      o->sector_in_file = k;
    }
  }
}

/* Every (disk sector, master sector) pair with a compatible position and equal
 * bytes, compared byte by byte with no signature at all. Lexicographic order. */
int64_t oracle_bruteforce(const uint8_t* image, uint64_t n_bytes, const uint8_t* masters,
                          const uint64_t* file_offsets, uint32_t n_files, uint32_t tau0, int any_tau,
                          oracle_match* out, uint64_t cap, int threads) {
  if (threads < 1) threads = 1;
  uint64_t n = n_bytes / SECTOR_BYTES;
  brute_ctx c = {image, masters, file_offsets, n_files, tau0, any_tau, NULL, NULL, NULL};
  c.part = (oracle_match**)calloc(threads, sizeof(oracle_match*));
  c.part_n = (uint64_t*)calloc(threads, sizeof(uint64_t));
  c.part_cap = (uint64_t*)calloc(threads, sizeof(uint64_t));
  parallel_for(n, threads, brute_range, &c);
  uint64_t cnt = 0;
  for (int t = 0; t < threads; t++) {
    for (uint64_t i = 0; i < c.part_n[t]; i++) {
      if (cnt < cap) out[cnt] = c.part[t][i];
      cnt++;
    }
    free(c.part[t]);
  }
  free(c.part);
  free(c.part_n);
  free(c.part_cap);
  return (int64_t)cnt;
}

/* ---------------------------------------------- fragments (Section 5) */
static uint64_t n_windows(uint64_t n_bytes) {
  return n_bytes < FRAGMENT_BYTES ? 0 : (n_bytes - FRAGMENT_BYTES) / WINDOW_STRIDE + 1;
}

typedef struct {
  const oracle_index* ix;
  const uint8_t* image;
  uint8_t* flag;
} window_ctx;

static void window_range(void* p, uint64_t lo, uint64_t hi, int t) {
  (void)t;
  window_ctx* c = (window_ctx*)p;
  for (uint64_t j = lo; j < hi; j++) {
    uint64_t h = signature_n(c->ix->sig_kind, c->image + j * WINDOW_STRIDE, FRAGMENT_BYTES);
    c->flag[j] = (uint8_t)is_flagged(c->ix, h, 0, 0, 1);
  }
}

/* Ascending ids j of the windows (bytes [4j, 4j + 64)) whose signature is
 * that of a master fragment. Returns the count; writes at most cap. */
int64_t oracle_fragment_flags(void* p, const uint8_t* image, uint64_t n_bytes, uint64_t* out, uint64_t cap,
                              int threads) {
  uint64_t n = n_windows(n_bytes);
  uint8_t* flag = (uint8_t*)malloc(n ? n : 1);
  window_ctx c = {(const oracle_index*)p, image, flag};
  parallel_for(n, threads, window_range, &c);
  uint64_t cnt = 0;
  for (uint64_t j = 0; j < n; j++)
    if (flag[j]) {
      if (cnt < cap) out[cnt] = j;
      cnt++;
    }
  free(flag);
  return (int64_t)cnt;
}

/* For each flagged window (ascending ids), every master fragment with an
 * equal signature and equal 64 bytes, in master order. */
int64_t oracle_fragment_confirm(void* p, const uint8_t* image, const uint64_t* ids, uint64_t n, oracle_match* out,
                                uint64_t cap) {
  const oracle_index* ix = (const oracle_index*)p;
  uint64_t cnt = 0;
  for (uint64_t i = 0; i < n; i++) {
    const uint8_t* w = image + ids[i] * WINDOW_STRIDE;
    uint64_t h = signature_n(ix->sig_kind, w, FRAGMENT_BYTES);
    for (uint64_t q = lower_bound(ix, h); q < ix->n && ix->e[q].sig == h; q++) {
      const oracle_entry* e = &ix->e[q];
      if (memcmp(w, ix->masters + e->master * FRAGMENT_BYTES, FRAGMENT_BYTES) != 0) continue;
      if (cnt < cap) {
        out[cnt].disk_sector = ids[i];
        out[cnt].file_id = e->file;
        out[cnt].sector_in_file = e->k;
      }
      cnt++;
    }
  }
  return (int64_t)cnt;
}

/* Every (window, master fragment) pair with equal bytes, compared byte by
 * byte with no signature. Window order, then master order. */
int64_t oracle_fragment_bruteforce(const uint8_t* image, uint64_t n_bytes, const uint8_t* fragments,
                                   const uint64_t* file_offsets, uint32_t n_files, oracle_match* out, uint64_t cap) {
  uint64_t n = n_windows(n_bytes);
  uint64_t n_m = n_files ? file_offsets[n_files] : 0;
  uint64_t cnt = 0;
  for (uint64_t j = 0; j < n; j++) {
    uint32_t f = 0;
    for (uint64_t m = 0; m < n_m; m++) {
      while (f + 1 < n_files && file_offsets[f + 1] <= m) f++;
      if (memcmp(image + j * WINDOW_STRIDE, fragments + m * FRAGMENT_BYTES, FRAGMENT_BYTES) != 0) continue;
      if (cnt < cap) {
        out[cnt].disk_sector = j;
        out[cnt].file_id = f;
        out[cnt].sector_in_file = (uint32_t)(m - file_offsets[f]);
      }
      cnt++;
    }
  }
  return (int64_t)cnt;
}
