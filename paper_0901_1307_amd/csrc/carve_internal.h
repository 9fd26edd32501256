// Library-internal entry points shared by carve.hip and carve_server.hip
// (hidden: not part of the C ABI).
#pragma once
#include <stdint.h>

#include "../../include/carve.h"

#define CARVE_HIDDEN extern "C" __attribute__((visibility("hidden")))

// Records a message for carve_last_error() and returns `code`.
CARVE_HIDDEN int carve_fail_msg(int code, const char* msg);

// Bytes per master unit of an index: 512 (sectors) or 64 (fragments).
CARVE_HIDDEN uint32_t carve_index_unit_bytes(const carve_index* idx);

// Creates *io when null and grows its device workspace (scan, compaction,
// confirmation, descriptors) for batches of up to n_sectors sectors in up to
// n_images images, so later scan_batch / batch_confirm_enqueue calls of that
// size allocate nothing (allocation and freeing synchronize the device).
CARVE_HIDDEN int carve_batch_reserve(const carve_index* idx, carve_batch** io, uint64_t n_sectors,
                                     uint32_t n_images, void* stream);

// Host-visible destinations of one batch's results (pinned memory).
struct carve_stage_out {
  uint64_t* totals;           // [0] flagged sectors, [1] confirmed matches (0 without confirmation)
  uint64_t* img_off;          // n_images + 1: first id of each image; [n] = flagged total
  uint64_t* ids;              // flagged ids, all images in order: min(flagged, ids_cap) written
  uint64_t ids_cap;
  carve_batch_match* matches; // records in image order: min(matches, staged room, match_cap) written
  uint64_t match_cap;
};

// Enqueues, on the batch's stream behind its scan (and its confirmation when
// `with_matches`), one kernel that writes the totals, the per-image offsets,
// the ids and the records into `st`. Nothing waits: once the stream reaches
// this point the host reads `st`. Results larger than a capacity are
// truncated there; *match_room receives how many records the device holds
// (more matches than that must be fetched with batch_confirm_matches).
CARVE_HIDDEN int carve_batch_stage_out(carve_batch* b, int with_matches, const carve_stage_out* st,
                                       uint64_t* match_room);

// Scan blocks per CU for a batch object's later launches (0: the index's
// setting), and how many blocks per CU the batch scan kernel can keep resident.
// The server gives a lane that starts while another lane runs half the CUs'
// slots, so the two lanes' persistent grids are resident together.
CARVE_HIDDEN int carve_batch_set_grid(carve_batch* b, uint32_t blocks_per_cu);
CARVE_HIDDEN uint32_t carve_batch_scan_blocks_per_cu(void);
