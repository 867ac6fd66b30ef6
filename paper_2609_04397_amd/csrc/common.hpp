// Internal definitions shared by the host planner, the ABI layer and the
// gfx950 kernels of the variable-block sparse library.
#pragma once

#include <algorithm>
#include <array>
#include <atomic>
#include <exception>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

namespace vbcsr {

// One block row ("panel") of one direction of the operator.
//
// The forward direction stores block row i of A as a dense b_i x K_i panel,
// K_i = sum of b_j over its stored blocks, column-major: panel element (p, k)
// sits at vbase + k*b + p.  Blocks keep their identity: block (i, j) fills
// the contiguous panel columns [k0, k0 + b_j), i.e. a contiguous run of
// b_i*b_j values holding the block column-major.  Inside a row, blocks are
// ordered by (b_j, j), so each shape class (b_i, b_j) of the row is one
// contiguous run.  The transposed direction stores A^T the same way, so its
// blocks are the untransposed source blocks, row-major.
struct RowDesc {
  int64_t vbase;  // first value of the panel (elements of the page type)
  int64_t cbase;  // first entry of the panel in the column table
  int32_t K;      // panel width (scalar columns)
  int32_t yrow;   // first output scalar row (off_i)
  int32_t b;      // panel height (b_i)
  int32_t pad;
};
static_assert(sizeof(RowDesc) == 32, "RowDesc layout");

// Value pages: every panel starts at a multiple of this many values; the
// gap after a panel holds zeros.  FP64/FP32 pages are followed by
// kPageSlack zero values.
constexpr int64_t kPanelAlign = 4;
constexpr int64_t kPageSlack = 2;

// Run body(r0, r1) over chunks of 512 rows of [0, n) on up to 16 threads
// (one thread when n is below 8192).  A thread that cannot be started leaves
// its share to the others; an exception thrown by body stops the remaining
// chunks and is rethrown here once every thread has joined.
template <typename F>
inline void parallel_rows(int32_t n, F &&body) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 8192) nt = 1;
  const int64_t chunk = 512;
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&]() {
    try {
      for (;;) {
        const int64_t r0 = next.fetch_add(chunk);
        if (r0 >= n) break;
        body((int32_t)r0, (int32_t)std::min<int64_t>(n, r0 + chunk));
      }
    } catch (...) {
      std::lock_guard<std::mutex> lock(mu);
      if (!err) err = std::current_exception();
      next.store(n);
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) {
    try {
      th.emplace_back(work);
    } catch (...) {
      break;
    }
  }
  work();
  for (auto &x : th) x.join();
  if (err) std::rethrow_exception(err);
}

// A std::vector whose new elements are left uninitialised: large host
// buffers are then first written (and paged in) by the threads that fill
// them instead of being zeroed by one thread.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U> &) {}
  template <typename U, typename... Args>
  void construct(U *p, Args &&...args) {
    if constexpr (sizeof...(Args) == 0)
      ::new (static_cast<void *>(p)) U;
    else
      ::new (static_cast<void *>(p)) U(std::forward<Args>(args)...);
  }
};
template <typename T>
using RawVec = std::vector<T, NoInitAlloc<T>>;

struct DirPlan {
  std::vector<RowDesc> rows;     // one per atom, in processing order
  std::vector<int32_t> colx;     // per panel column: scalar row of the input vector
  std::vector<int64_t> colg;     // forward only, per panel column: (graph offset of the
                                 // column's block + q) << 7 | b_j (block-sampled product)
  RawVec<int64_t> blk_pos;       // per graph block: page offset of its first value
  RawVec<int32_t> blk_k0;        // per graph block: first panel column
  RawVec<int32_t> blk_prow;      // per graph block: index (processing order) of its panel
  std::vector<int64_t> vbase16;  // per panel (processing order): offset in the BF16 pages
  int64_t n_values = 0;          // values in the pages
  int64_t n_values16 = 0;        // values in each BF16 page (panels padded to 8 columns)
  int64_t n_cols = 0;            // entries of the column table
};

struct HostPlan {
  int32_t n = 0;        // atoms (block columns; block rows of a square operator)
  int32_t n_rows = 0;   // block rows that may hold blocks: n, or the owned atoms
                        // of a rank-local operator (the first n_rows atoms)
  int64_t N = 0, N_rows = 0, nnzb = 0, nnz = 0;
  std::vector<int64_t> off;                   // n+1 scalar row offsets
  RawVec<int64_t> gbase;                      // nnzb+1 graph value offsets
  RawVec<int32_t> blk_row;                    // per graph block: block row i
  std::vector<std::array<int32_t, 3>> shapes; // (b_i, b_j, count), ascending
  DirPlan fwd, tr;
};

// Host-side validation of a block graph; returns a VBCSR_* status and fills
// `err` on failure.  Touches no device.
int validate_graph(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                   int64_t n_values, std::string &err);

// Build both directions of the plan (assumes validate_graph passed).  With
// with_columns unset the column tables (colx, colg) are left empty and only
// their sizes (n_cols) are set; the device builds them from the per-block
// maps (blk_prow, blk_k0).  n_rows >= 0 (rank-local operators): only atoms
// below n_rows hold blocks in their rows; the forward direction then has
// n_rows panels and the transposed one n (default: n_rows = n).
void build_plan(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                int32_t row_order, HostPlan &plan, bool with_columns = true,
                int32_t n_rows = -1);


// Record `msg` as the calling thread's last error (read by vbcsr_last_error)
// and return `code`.
int set_error(int code, const std::string &msg);

// For a catch (...) around an entry point: the status of the exception in
// flight (ENOMEM for host allocation and thread-resource failures, EINVAL
// otherwise), with `where` and its message recorded as the last error.
int api_exception(const char *where);

}  // namespace vbcsr
