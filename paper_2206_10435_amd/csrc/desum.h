// Arguments of the expansion kernel: compacted summary arrays of every table,
// already offset to the table's slots.
#pragma once
#include "gj_internal.h"

namespace gjk {

struct DTab {
  const int32_t* perm;     // grouped row ids of the table
  const int64_t* cpre;     // surviving entry -> offset of its block inside its group (units of c*U)
  const int2* ccs;         // surviving entry -> (row count, first position in perm)
  const ChildRec* crec;    // (t >= 1) surviving parent entry -> this table's group
  const int64_t* cU;       // surviving entry -> U (the group message is cpre + c*U at its last entry)
  int32_t parent;
};

struct DesumArgs {
  DTab tab[GJ_MAX_TABLES];
  int64_t first;   // rank of the first tuple
  int64_t n_rows;  // tuples to write
  int64_t n_root;  // surviving root entries
  void* out;
  int32_t n_tables;
  int32_t k_round;
  int32_t tuples_per_lane;
  // value columns (n_cols = 0: row ids of every table): column j is
  // col_src[j][position of table col_tab[j]'s row in its grouped order]
  int32_t n_cols;
  int32_t col_tab[GJ_MAX_OUT_COLS];
  const int32_t* col_src[GJ_MAX_OUT_COLS];
};


// LDS of an expansion block: every lane stages a round of ks tuples of nc
// values of wbytes each (whole 16-byte units) in a slot of the next power of
// two of units, or (tight) of exactly its units when that is not a power of
// two (row-id launches: less LDS per wave, more waves per CU).
inline size_t staging_bytes(int ks, int nc, int wbytes, bool tight = false) {
  const int upl = ks * nc * wbytes / 16;
  int p = 1;
  while (p < upl) p <<= 1;
  return (size_t)GJ_BLOCK * (tight ? upl : p) * 16;
}

// Arguments of the run expansion of a projected summary (desum_runs.hip).
struct RunTab {
  const int64_t* cpre;    // surviving entry -> offset of its block inside its group (units of c*U)
  const int64_t* cc;      // surviving entry -> frequency c (int64)
  const ChildRec* crec;   // (t >= 1) surviving parent entry -> this table's group
  const int64_t* cU;      // surviving entry -> U (the group message is cpre + c*U at its last entry)
  int32_t parent;
};

struct RunArgs {
  RunTab tab[GJ_MAX_TABLES];
  int64_t first, n_rows, n_root;
  int32_t* out;  // row-major [n_rows x n_cols] int32
  int32_t n_tables, n_cols, tuples_per_lane;
  int32_t col_tab[GJ_MAX_OUT_COLS];         // table of result column j
  const int32_t* col_key[GJ_MAX_OUT_COLS];  // its key column, by surviving entry
};

}  // namespace gjk
