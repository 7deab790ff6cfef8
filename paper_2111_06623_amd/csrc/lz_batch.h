// Work-list launches: one launch of a kernel over the blocks of several
// instances (the batched q sweep and the uneven batch advance their
// recursions with one launch per stage instead of one per stage and
// instance).
//
// Every kernel of a Lanczos step takes its arguments as one struct P and a
// BatchRef.  With a null item table the launch is an ordinary one: P is the
// kernel argument and the block index is the hardware's.  Otherwise block b
// of the launch is work item item[b]: instance i = item[b] >> 24 and the
// linear block index l = item[b] & 0xFFFFFF of that instance's own grid (x
// fastest).  Instance i's record sits at tab + i * stride: its grid
// (BatchGrid), then its argument struct P.  Each instance keeps its own sizes,
// buffers and launch configuration; only the kernel (and so the block shape)
// is common to a merged launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

namespace lz {

struct BatchRef {
  const unsigned char* tab;  // instance records (BatchGrid + argument struct)
  const unsigned* item;      // one entry per block of the launch; null: ordinary launch
  int stride;                // bytes per instance record
  int pad;
};

struct BatchGrid {
  int x, y, z, pad;
};

// block index and grid of the block being run (the instance's own)
struct VBlock {
  int x, y, z;
  int nx, ny, nz;
};

constexpr int kBatchMaxInst = 256;
constexpr unsigned kBatchLocalMask = (1u << 24) - 1u;

template <class P>
__device__ __forceinline__ const P& batch_args(const BatchRef& br, VBlock& vb) {
  const unsigned e = br.item[blockIdx.x];
  const unsigned char* rec = br.tab + (size_t)(e >> 24) * br.stride;
  const BatchGrid g = *reinterpret_cast<const BatchGrid*>(rec);
  int l = (int)(e & kBatchLocalMask);
  vb.nx = g.x;
  vb.ny = g.y;
  vb.nz = g.z;
  vb.x = l % g.x;
  l /= g.x;
  vb.y = l % g.y;
  vb.z = l / g.y;
  return *reinterpret_cast<const P*>(rec + sizeof(BatchGrid));
}

__device__ __forceinline__ VBlock native_block() {
  return VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z,
                (int)gridDim.x,  (int)gridDim.y,  (int)gridDim.z};
}

// Kernel entry: CALL runs with `a_` bound to the block's argument struct and
// `vb` to its block index: from the kernel argument P and the hardware's
// block index (BAT false, the ordinary kernel), or from the work-item table BR
// (BAT true, the kernel's work-list twin, compiled separately so that the
// ordinary kernel's code and registers are those of a plain kernel).
#define LZ_BATCHED(BAT, P, BR, CALL)                                      \
  do {                                                                    \
    if constexpr (BAT) {                                                  \
      VBlock vb;                                                          \
      const auto& a_ = batch_args<decltype(P)>((BR), vb);                 \
      CALL;                                                               \
    } else {                                                              \
      const VBlock vb = native_block();                                   \
      const auto& a_ = (P);                                               \
      CALL;                                                               \
    }                                                                     \
  } while (0)

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// A launch as issued by one instance: kernel, its work-list twin, grid,
// block shape, dynamic LDS and the bytes of its argument struct.
struct LaunchRec {
  const void* fn;
  const void* fnb;
  dim3 grid, block;
  size_t lds;
  std::vector<unsigned char> args;
};

// While non-null, launches of this thread are appended here instead of being
// issued (lz_api.hip records the launch sequence of a step per instance and
// merges the sequences of instances that issue the same kernels).
extern thread_local std::vector<LaunchRec>* t_launch_rec;

// Issue fn (a kernel k(P, BatchRef)) as an ordinary launch with the argument
// bytes p, or record it with its twin fnb; throws std::runtime_error when HIP
// refuses the launch.
void launch_args(const void* fn, const void* fnb, dim3 grid, dim3 block, size_t lds,
                 hipStream_t s, const void* p, size_t bytes);

template <class P, class... A>
inline void lz_launch(void (*fn)(P, BatchRef), void (*fnb)(P, BatchRef), dim3 grid, dim3 block,
                      size_t lds, hipStream_t s, A&&... a) {
  const P p{std::forward<A>(a)...};
  launch_args(reinterpret_cast<const void*>(fn), reinterpret_cast<const void*>(fnb), grid, block,
              lds, s, &p, sizeof(P));
}

}  // namespace lz
