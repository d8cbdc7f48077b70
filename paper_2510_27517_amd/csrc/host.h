// Host-side building blocks of the library: CSR validation and transpose,
// rounding to the half storage formats, preconditioner construction, and the
// row-block partition used by the kernels. No GPU calls.
#pragma once
#include <climits>
#include <cstdint>
#include <string>
#include <vector>

namespace pcgh {

// PCG_OK or PCG_EINVAL (with a reason in *why when given).
int validate_csr(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, int require_diag, std::string *why);

// CSR of the transpose of an n x n matrix (stable: rows of the transpose list
// the original rows in ascending order).
void transpose_csr(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                   const std::vector<double> &v, std::vector<int32_t> &trp, std::vector<int32_t> &tci,
                   std::vector<double> &tv);

// Round to nearest, ties to even, onto the BF16 / FP16 grids (bit patterns).
uint16_t to_bf16_bits(double v);
uint16_t to_f16_bits(double v);

// Nonzeros of G for a preconditioner kind on A's pattern (-1: unknown kind).
int64_t g_nnz(int kind, int32_t n, const int32_t *rp, const int32_t *ci);

// CPUs this process may run on (its affinity mask), at least 1.
unsigned available_cpus();

// G (CSR) for a preconditioner kind built from A (seed: PCG_G_SEEDED). The
// FSAI rows are built on `threads` threads (0: available_cpus(), at most 32;
// systems too small to pay for threads use one).
int build_g(int kind, uint64_t seed, int32_t n, const int32_t *rp, const int32_t *ci, const double *v, std::vector<int32_t> &grp,
            std::vector<int32_t> &gci, std::vector<double> &gv, int threads = 0);

// Row-block partition: (row start, nonzero start) pairs, nblk + 1 of them.
std::vector<int32_t> row_blocks(int32_t n, const int32_t *rp, int cap);

// Sliced ELL with slices of kSlice consecutive rows: slice c holds
// so[c+1] - so[c] columns (its longest row); entry k of row 64c + l sits at
// (so[c] + k) * kSlice + l. Rows keep their CSR order; shorter rows and rows
// past n are padded with column `pad_col(row)` and value 0.
constexpr int kSlice = 64;

// Stored entries (nonzeros plus padding) of the sliced layout of a pattern.
int64_t sell_entries(int32_t n, const int32_t *rp);

// Slice offsets: nslice + 1 of them, in units of kSlice entries.
void sell_offsets(int32_t n, const int32_t *rp, std::vector<int32_t> &so);

// Columns in sliced order; a padding entry takes its own row as column (0
// for rows past n), so every gather stays in range.
void sell_columns(int32_t n, const int32_t *rp, const int32_t *ci, const std::vector<int32_t> &so,
                  std::vector<int32_t> &out);

// Elements of `esz` bytes in CSR order (`in`) moved to sliced order; padding
// is all-zero bytes (+0 in every floating-point format).
void sell_bytes(int32_t n, const int32_t *rp, const uint8_t *in, size_t esz, const std::vector<int32_t> &so,
                std::vector<uint8_t> &out);

// Sliced diagonal layout (SDIA): slices of kSlice rows as in sliced ELL, but
// the column of an entry is stored once per slice as its offset from the
// row: slice c lists the distinct offsets (column - row) of its entries in
// ascending order, offs[so[c] .. so[c+1]), and stores for every row one value
// per listed offset, at (so[c] + k) * kSlice + l for row kSlice c + l (0 where
// the row has no entry at that offset; rows past n hold zeros). Each row's
// values stay in ascending column order, the CSR order, with zeros between.
// Good for stencil and banded matrices, where a slice's rows share offsets.

// Stored values (kSlice per listed offset) of the SDIA layout of a pattern;
// the count stops growing past `stop` (it is then only known to exceed it).
int64_t sdia_entries(int32_t n, const int32_t *rp, const int32_t *ci, int64_t stop = INT64_MAX);

// Slice offsets into offs (nslice + 1, in units of listed offsets) and the
// listed offsets, slice by slice.
void sdia_pattern(int32_t n, const int32_t *rp, const int32_t *ci, std::vector<int32_t> &so,
                  std::vector<int32_t> &offs);

// Elements of `esz` bytes in CSR order moved to the SDIA order (all other
// bytes zero).
void sdia_bytes(int32_t n, const int32_t *rp, const int32_t *ci, const uint8_t *in, size_t esz,
                const std::vector<int32_t> &so, const std::vector<int32_t> &offs, std::vector<uint8_t> &out);

// Sliced 3x3-block layout: the matrix is exactly 3x3-blocked when n % 3 == 0
// and rows 3R, 3R+1, 3R+2 store the same columns, all in complete groups
// {3C, 3C+1, 3C+2}. Slices of kBSlice block rows (3 kBSlice rows, one lane
// each); slice c holds bo[c+1] - bo[c] blocks per block row (its longest
// block row); block k of block row kBSlice c + r has column index
// bcol[(bo[c] + k) kBSlice + r]. Its row s, column j value sits, for 8-byte
// values, at ((bo[c] + k) 3 + j) 3 kBSlice + s kBSlice + r (for each block
// and column the slice's rows are contiguous: one coalesced load per column),
// and for narrower values at 9 ((bo[c] + k) kBSlice + r) + 3 s + j (each row's
// three values contiguous, rows adjacent: one wide load per lane). Padding
// blocks take their own block row as column and zero values.
constexpr int kBSlice = 21;

// True when the pattern is exactly 3x3-blocked; *blocks = number of blocks.
bool is_block3(int32_t n, const int32_t *rp, const int32_t *ci, int64_t *blocks);

// Stored blocks (with padding) of the sliced block layout.
int64_t bsell_blocks(int32_t n, const int32_t *rp);

// Block offsets (nslice + 1) and block columns in sliced order.
void bsell_pattern(int32_t n, const int32_t *rp, const int32_t *ci, std::vector<int32_t> &bo,
                   std::vector<int32_t> &bcol);

// Elements of `esz` bytes in CSR order moved to the sliced block order
// (padding all-zero bytes).
void bsell_bytes(int32_t n, const int32_t *rp, const uint8_t *in, size_t esz, const std::vector<int32_t> &bo,
                 std::vector<uint8_t> &out);

// Algorithmic bytes of one PCG iteration (11 vector streams).
double bytes_per_iter(int32_t n, int64_t a, int64_t g, int adt, int gdt, int vdt);

}  // namespace pcgh
