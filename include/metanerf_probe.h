/*
 * metanerf_probe.h -- machine-ceiling probes.
 *
 * Not part of the rendering path: two micro-kernels that measure what the
 * GPU sustains for the two kinds of work the renderer is made of, so that
 * the renderer's rates can be read against measured ceilings as well as
 * the published peaks:
 *   - small random gathers from a table of the grid encoding's size
 *     (the warp and encoding steps, Sec. 4.2 Eq. 9 and Sec. 4.4 Eq. 13);
 *   - a dense MFMA loop in the MLP's arithmetic types (the MLP of Eq. 13);
 *   - scattered float atomics (the adjoint's gradient scatter, Sec. 5.2),
 *     in memory and in LDS (the adjoint's block sums);
 *   - the renderer's MLP run unfused, over features read from memory.
 * All run on the caller's stream; time them with events around the call.
 */
#ifndef METANERF_PROBE_H
#define METANERF_PROBE_H

#include "metanerf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Each of n_lanes lanes (a multiple of 256) reads gathers_per_lane (a
 * multiple of 8, >= 8) rows of row_bytes (4, 8 or 16) from the dev table of
 * table_bytes (row_bytes .. 2^31-1 bytes), eight loads in flight at a time,
 * and writes the float sum of what it read to out[lane] (dev float
 * [n_lanes]).  window_bytes = 0: rows uniform over the table.  Otherwise
 * the 64 lanes of a wave draw their rows from one window of that many bytes
 * (a fresh random window per gather), the access pattern of neighbouring
 * rays.  Row choice is a fixed hash of (seed, lane, k).  Gathers issued =
 * n_lanes * gathers_per_lane. */
mnr_status mnr_probe_gather(const void* table, uint64_t table_bytes, int32_t row_bytes, uint32_t window_bytes,
                            int32_t gathers_per_lane, int32_t n_lanes, uint32_t seed, float* out, void* stream);

/* Each of n_lanes lanes (a multiple of 256) adds 1.0f with
 * atomics_per_lane device-scope float atomics (no return value) to words of
 * the dev float buffer acc[n_words] chosen by a fixed hash of (seed, lane /
 * run, k): `run` consecutive lanes (1..64) share each address, the pattern
 * of consecutive samples of one ray in a coarse cell.  The adjoint's
 * scatter is made of such atomics.  Atomics issued = n_lanes *
 * atomics_per_lane; the buffer's sum grows by exactly that. */
mnr_status mnr_probe_atomic(float* acc, uint32_t n_words, int32_t atomics_per_lane, int32_t n_lanes, int32_t run,
                            uint32_t seed, void* stream);

/* LDS operations, the block sums of the adjoint: n_blocks blocks of 1024
 * threads (4..4096) each zero an LDS array of 8192 words (32 KiB per
 * type), then every thread performs `iters` (1..100000) operations on word
 * (thread + 97 k) mod 8192 (consecutive lanes on consecutive words, no two
 * lanes of a wave on one bank), op: 0 float atomic add, 1 32-bit integer
 * atomic add, 2 64-bit integer atomic add (4096 words), 3 plain float
 * read-add-write, 4 plain 32-bit store.  Lane operations issued =
 * n_blocks * 1024 * iters.  out: dev float [n_blocks * 1024] (each thread's
 * first word afterwards, so that nothing is optimised away). */
mnr_status mnr_probe_lds(int32_t op, int32_t iters, int32_t n_blocks, float* out, void* stream);

/* n_blocks blocks of 4 waves each run `iters` iterations of 4 independent
 * MFMA chains: F32 -> v_mfma_f32_16x16x4f32 (2048 FLOP each), BF16 ->
 * v_mfma_f32_16x16x32_bf16 (16384 FLOP each).  FLOP issued = n_blocks * 4
 * waves * iters * 4 * (FLOP per MFMA).  out: dev float [n_blocks * 256]. */
mnr_status mnr_probe_mfma(mnr_dtype dtype, int32_t iters, int32_t n_blocks, float* out, void* stream);

/* The field MLP of Sec. 4.4 Eq. 13 (the grid-encoded field's: 32 -> 64 ...
 * -> 4, bias-free, ReLU hidden layers) on its own, with the renderer's
 * device code: the weights field->w[] (field->mlp_dtype, F32 or BF16;
 * field->n_layers 2..4; other field members are not read) are staged into
 * LDS once per block, and each wave pushes 64-sample chunks through the
 * MFMA layer chain.  feat: dev [n][32] features in the MLP's type (F32:
 * float, BF16: bfloat16), 16-byte aligned.  out: dev float [n][4], 16-byte
 * aligned, receives (sigmoid(o0), sigmoid(o1), sigmoid(o2), ReLU(o3)), the
 * colour and density heads of Sec. 4.4.  n = 0 launches nothing.  Reads
 * 128 (F32) or 64 (BF16) bytes and writes 16 bytes per sample; MLP work
 * 2 * (32*64 + (n_layers-2)*64*64 + 64*4) FLOP per sample.  Errors: null
 * pointers, misalignment, widths other than 32/64/4, a frequency-encoded
 * field (MNR_E_UNSUPPORTED). */
mnr_status mnr_probe_mlp(const mnr_field* field, const void* feat, int64_t n, float* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* METANERF_PROBE_H */
