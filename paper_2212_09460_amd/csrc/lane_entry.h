// Internal entry points that one source file of liblane.so defines and
// others call, declared once: every file that defines or calls one includes
// this header, so a definition that drifts from its callers' view fails to
// compile instead of being linked by name (C linkage carries no types).
#pragma once

#include "../../include/lane.h"
#include "lane_internal.h"

extern "C" {

// sobel.hip
LANE_INTERNAL hipError_t lane_launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
LANE_INTERNAL hipError_t lane_launch_sobel(const lane::SobelDesc* d, int mode, hipStream_t s);
LANE_INTERNAL hipError_t lane_launch_sobel_batch(const lane::SobelDesc* descs, const int2* items,
                                                 const int* counts, int fast, int latency, int grid,
                                                 hipStream_t s);
LANE_INTERNAL int lane_sobel_items(int W, int H, int strip_rows);
LANE_INTERNAL int lane_sobel_fast_ok(const lane::SobelDesc* d, int mode);

// vote.hip, vote_pair.hip, prune.hip
LANE_INTERNAL hipError_t lane_launch_vote(const lane::VoteDesc* d, hipStream_t s);
LANE_INTERNAL hipError_t lane_launch_vote_batch(const lane::VoteDesc* descs, const int2* items,
                                                const int* n_items, uint32_t* queue, const int* xends,
                                                int half_lds, int grid, hipStream_t s);
LANE_INTERNAL hipError_t lane_launch_vote_pair(const lane::VoteDesc* d, int pairing, hipStream_t s);
LANE_INTERNAL hipError_t lane_launch_prune_batch(const lane::PruneDesc* descs, int n, int max_nseg,
                                                 hipStream_t s);

// peaks.hip
LANE_INTERNAL hipError_t lane_launch_peaks(const lane::PeaksDesc* d, hipStream_t s);
LANE_INTERNAL hipError_t lane_launch_peaks_batch(const lane::PeaksDesc* descs, const int* list,
                                                 const int* counts, int n_frames, int grid_keys,
                                                 int grid_select, hipStream_t s);

// lines.hip, canny.hip, progressive.hip
LANE_INTERNAL hipError_t lane_launch_lines(const uint8_t* edges, int W, int H, const int16_t* C,
                                           const int16_t* S, int n_theta, int r_offset,
                                           const int32_t* theta_idx, const int32_t* r_idx,
                                           const int32_t* count, int k, int fill_gap, int min_length,
                                           int max_seg, int32_t* segs, int32_t* seg_count,
                                           int32_t* npts, hipStream_t s);
LANE_INTERNAL hipError_t lane_launch_lines_batch(const lane::LinesDesc* descs, int n, int max_k,
                                                 int max_side, hipStream_t s);
LANE_INTERNAL size_t lane_canny_ws_bytes(int W, int H);
LANE_INTERNAL hipError_t lane_launch_canny(const uint8_t* img, int W, int H, int pitch, int t_low,
                                           int t_high, int border_mode, uint8_t* edges, uint8_t* mag,
                                           uint32_t* edge_count, void* ws, hipStream_t s);
LANE_INTERNAL hipError_t lane_launch_progressive(const lane::ProgDesc* d, const lane::PeaksDesc* pk,
                                                 hipStream_t s);

// capi.hip: layout rules shared with the plans
LANE_INTERNAL int lane_vote_row_cap(int32_t W, int32_t H, int32_t n_r);
LANE_INTERNAL long lane_vote_slice_words(int32_t W, int32_t H, int32_t n_theta, int32_t n_r, int T);
LANE_INTERNAL int lane_vote_rows_per_group(int32_t W, int32_t H, int32_t n_theta, int32_t n_r);
LANE_INTERNAL int lane_vote_rows_default(int32_t W, int32_t H, int32_t n_theta, int32_t n_r);
LANE_INTERNAL int lane_peaks_block_log2(int32_t n_theta, int32_t n_r);
LANE_INTERNAL int lane_peaks_blocks_per_row(int32_t n_r, int lg);
LANE_INTERNAL int lane_peaks_prepare(const int32_t* acc, int32_t n_theta, int32_t n_r, int32_t r_offset,
                                     int32_t k, int32_t h_theta, int32_t h_r, int32_t min_votes,
                                     int32_t* theta_idx, int32_t* r_idx, int32_t* votes, int32_t* count,
                                     lane::PeaksDesc* d, size_t* need);

// cnn.hip: forward and inference with per-frame switches, masks
LANE_INTERNAL int lane_cnn_forward_active(const uint8_t* img, int32_t W, int32_t H, int32_t pitch,
                                          int64_t img_stride, int32_t batch, const void* packed,
                                          void* act, float* logits, const uint8_t* active,
                                          void* stream);
LANE_INTERNAL int lane_cnn_infer_mask_active(const uint8_t* img, int32_t W, int32_t H, int32_t pitch,
                                             int64_t img_stride, int32_t batch, const void* packed,
                                             float* logits, float conf, uint8_t* mask,
                                             const uint8_t* active, void* stream);
LANE_INTERNAL int lane_cnn_infer_active(const uint8_t* img, int32_t W, int32_t H, int32_t pitch,
                                        int64_t img_stride, int32_t batch, const void* packed,
                                        float* logits, const uint8_t* active, void* stream);
LANE_INTERNAL int lane_mask_from_logits_active(const float* logits, int32_t W, int32_t H,
                                               int32_t batch, float conf, uint8_t* mask,
                                               const uint8_t* active, void* stream);

// batch.hip
LANE_INTERNAL int lane_batch_create_shaped(const lane_frame* frames, int32_t n, const lane_tune* tune_opt,
                                           int latency, lane_batch** out);
LANE_INTERNAL int lane_batch_enqueue_pass_stage(lane_batch* b, int32_t stage, void* stream);

}  // extern "C"
