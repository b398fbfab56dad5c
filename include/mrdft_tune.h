/*
 * mrdft_tune.h — persistent cache of tuned forward schedules (part of
 * libmrdft.so; host code only, usable without a GPU).
 *
 * Not part of the paper: the paper's scheme (Section 3, eq. (4)) fixes the
 * arithmetic, not the order in which a GPU runs it.  The library picks a
 * schedule (on-chip tile depth, job order, persistent grid, whether the levels
 * above the tile run on side streams) by timing candidates when a plan is
 * created with MRDFT_FLAG_TUNE; this cache keeps those choices across
 * processes.
 *
 * File format: one JSON object, versioned,
 *   {"format": "mrdft-tune", "version": 1,
 *    "entries": {"<key>": {"tile_log": T, "grid": G, "order": O, "serial": S}, ...}}
 * with non-negative integers T, G, O, S (S: 0 side streams beside the main
 * launch, 1 every launch on the caller's stream, 2 side streams after it).  A file that does not parse, has
 * another format name or version, or holds an entry with a missing or
 * negative field is treated as empty (never an error): lookups miss and the
 * next store replaces it with a valid file.
 *
 * Keys are built by the library from the device architecture name, the input
 * type, the output form and the shape of the batch; any string without
 * control characters, '"' or '\\' is accepted.
 *
 * Return values are mrdft_status codes (include/mrdft.h): 0 = MRDFT_OK,
 * 1 = MRDFT_E_INVALID_ARG, 3 = MRDFT_E_ALLOC.  Calls on one file from several
 * threads or processes are safe in the sense that the file is always replaced
 * whole (write to a temporary file, then rename); the last store wins.
 */
#ifndef MRDFT_TUNE_H
#define MRDFT_TUNE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Version of the file format written and accepted. */
#define MRDFT_TUNE_CACHE_VERSION 1

/*
 * Look up `key` in the cache file `path` (host strings, NUL-terminated).
 * Returns 1 and writes the four values on a hit; returns 0 on a miss,
 * including a missing, unreadable or corrupt file.  Returns -1 if an argument
 * is NULL or the key is not acceptable.  Output pointers are written only on
 * a hit.
 */
int mrdft_tune_cache_lookup(const char* path, const char* key, int* tile_log, int* grid, int* order, int* serial);

/*
 * Insert or replace `key` in `path`, keeping every other valid entry of the
 * existing file (a corrupt file is replaced).  Values must be >= 0.
 * Returns 0 (MRDFT_OK), 1 (MRDFT_E_INVALID_ARG: NULL argument, bad key,
 * negative value) or 3 (MRDFT_E_ALLOC: the file could not be written).
 */
int mrdft_tune_cache_store(const char* path, const char* key, int tile_log, int grid, int order, int serial);

#ifdef __cplusplus
}
#endif
#endif /* MRDFT_TUNE_H */
