// Internal declarations shared by the host driver (mr_grid.cpp) and the HIP
// kernels (mr_device.hip).  Not part of the public ABI (include/mr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mr {

// Zero-detail refinement of a box (coarse-extension assumption, section
// 2.2.2): the tensor Deslauriers-Dubuc refinement of the level-(L-1) samples
// around a box of level-L points of block blk.  A patch item covers the
// coarser regions of blk on one side (bit r of rmask set for region r);
// each point is written into the patch of its region.  A substitution item
// (sections 2.2.4, 2.3) is a box of blk's slabs next to coarser leaves; the
// kernel replaces the box's slab points degree by degree.
struct GItem {
  int32_t blk;      // fine block whose owner map resolves the samples
  int32_t sel;      // bit 3 = lifted wavelet, bit 4 = substitution item
  int32_t lo[3];    // box [lo, hi) of level-L points, relative to blk's
  int32_t hi[3];    //   origin at blk's level
  int32_t rmask;    // patch item: regions (rx + 3 ry + 9 rz) written
  int32_t pad;
};

// Restriction of finer data to coarse ghost points (f->c, ghosting Part 2):
// a fine block F coarsens its ghost-filled level-L field ([H^a]^3; injection
// for N.0) at the level-(L-1) points that lie in the ghost region of its
// coarser neighbour C, and writes them into C's patch.  Inside the
// restriction window, points held by leaves finer than F are injected.
struct RItem {
  int32_t fblk;     // fine block F
  int32_t cblk;     // coarse block C
  int32_t lo[3];    // output box, C-relative coordinates at C's level
  int32_t hi[3];
  int32_t sh[3];    // F-relative coarse coordinate = C-relative - sh
  int32_t rlo[3];   // C's patch region origin / extent
  int32_t rsz[3];
  int32_t pad;
  int64_t off;      // C's patch offset
};

// One separable pass of a box operation used by adaptation (refine, coarsen,
// update): out[box] = sum_o w(o) in[p + o*axis], where the 1D filter depends
// on the parity of the output coordinate along `axis`.
struct PItem {
  int32_t src_blk;  // block whose ext field / owner map the pass reads
  int32_t dst_blk;  // destination block in the destination field array
  int32_t lo[3];    // output box (relative coordinates of the pass output)
  int32_t hi[3];
  int32_t ilo[3];   // scratch input box origin / extent (src_mode 1)
  int32_t isz[3];
  int32_t dlo[3];   // field destination: block-local = output - dlo
  int32_t pad;
  int64_t in_off;   // scratch offset of the input box
  int64_t out_off;  // scratch offset of the output box (dst_mode 0)
};

enum Filter1D : int32_t {
  F_REFINE = 0,     // zero-detail synthesis (DD at odd, copy at even)
  F_RESTRICT = 1,   // H^a at even fine positions (output at coarse points)
  F_SYNTH = 2,      // J^s / K^s synthesis of an interleaved array
  F_ANALYSIS = 3    // H^a / G^a analysis (interleaved output)
};

// Device view of the grid.
template <typename T>
struct DevGrid {
  int32_t nb;
  int32_t nblk;
  const int32_t* lev;    // [nblk]
  const int32_t* ijk;    // [3*nblk]
  const int32_t* cmap;   // [64*nblk] leaf id per half-block cell of the
                         //   4x4x4 cells covering [-nb/2, 3nb/2)^3
  const int64_t* poff;   // [27*nblk] patch offset per region, -1 if none
  const uint64_t* stab;  // [8*nblk] slab table of each block (k_subst)
  const int64_t* cbase;  // [64*nblk] coarse-sample address table per cell
  const int32_t* cstep;  //   (see k_cell_tables)
  T* field;              // [nblk * nb^3]
  T* patch;
  int32_t dw;            // allocated depth of every patch region
  int32_t* err;          // device error counter (unsupported geometry)
};

struct VelDev {
  int32_t kind;
  double p[8];
};

struct IcDev {
  int32_t kind;
  int32_t n;
  const double* params;  // device pointer
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s`; T is float or double selected by `f32`.
struct Wavelet {
  int32_t N, Nt;
};

void launch_gview(bool f32, const void* dg, Wavelet w, const GItem* items, int n_items,
                  int lds_bytes, hipStream_t s);
void launch_subst(bool f32, const void* dg, Wavelet w, const GItem* items, int n, int lds,
                  int threads, hipStream_t s);
void launch_cell_tables(bool f32, const void* dg, int n_blocks, hipStream_t s);
void launch_rview(bool f32, const void* dg, Wavelet w, const RItem* items, int n_items,
                  int lds, int maxq, hipStream_t s);
// RK3 stage: out = a*un + b*(c*y + dt*rhs(y)) (c = 1 for the RK stages).
void launch_rhs(bool f32, const void* dg_y, const void* un, void* out, int fd_order, int depth,
                double a_un, double b_y, double c_y, double dt, const VelDev& vel, int first_blk,
                int n_blk, hipStream_t s);
// Details: per-block band maxima (27 per block, FP64), optional full detail
// array of selected blocks (det_slot[b] >= 0) into det_out.
void launch_details(bool f32, const void* dg, Wavelet w, int ef, int eb, double* bands,
                    const int32_t* det_slot, double* det_out, int first_blk, int n_blk,
                    hipStream_t s);
void launch_combine(const void* dg_any, const double* bands, int detail_ext, double* norms,
                    int n_blk, hipStream_t s);
void launch_sample_ic(bool f32, const void* dg, const IcDev& ic, hipStream_t s);
void launch_ic_error(bool f32, const void* dg, const IcDev& ic, double* out, hipStream_t s);
void launch_moments(bool f32, const void* dg, double* out, hipStream_t s);  // 4 per block
void launch_gather_ext(bool f32, const void* dg, int depth, int64_t b0, int64_t nblk, void* out,
                       hipStream_t s);
void launch_copy_blocks(bool f32, const void* src, void* dst, const int32_t* pairs, int n_pairs,
                        int nb, hipStream_t s);
void launch_fill(bool f32, void* dst, size_t n, hipStream_t s);
// src_mode: 0 gather the ext field of src_blk, 1 FP64 scratch box (din),
// 2 discarded details (det, det_slot per old block, det_tab: per slot 16
// words of 32 bits, bit (front | back << 3 | parity << 6) set when the
// slot's details with that per-axis slab membership and parity are
// discarded); dst_mode: 0 FP64 scratch box (dout), 1 store into dst field
// block, 2 subtract from dst field block (block-local coordinates = output -
// dlo).
void launch_pass(bool f32, const void* dg, Wavelet w, int filter, int axis, int src_mode,
                 int dst_mode, const PItem* items, int n_items, const double* din, double* dout,
                 const double* det, const int32_t* det_slot, const uint32_t* det_tab, void* dst,
                 hipStream_t s);

// Direction mask of a coarsening child's slot: all its details are discarded.
constexpr int32_t kDiscardAll = 1 << 27;
// Device address (current device) of the static band-maxima scratch of
// mr_details_noalloc, resolved once per device; its capacity in blocks.
hipError_t static_band_scratch(double** out);
int64_t static_band_blocks();
// Events to be stamped at the start and end of the next launch (NULL: none).
void set_launch_events(hipEvent_t start, hipEvent_t stop);

}  // namespace mr
