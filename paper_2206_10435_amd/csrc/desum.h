// Arguments of the expansion kernel: compacted summary arrays of every table,
// already offset to the table's slots.
#pragma once
#include "gj_internal.h"

namespace gjk {

struct DTab {
  const int32_t* perm;    // grouped row ids of the table
  const int64_t* cc;      // surviving entries: row count
  const int32_t* cstart;  // first position of the entry's rows in perm
  const int64_t* cpre;    // offset of the entry's block inside its group (units of c*U)
  const int32_t* clink;   // (t >= 1) surviving parent entry -> surviving group of t
  const int32_t* cglo;    // (t >= 1) surviving group -> first surviving entry
  const int32_t* cghi;    // (t >= 1) surviving group -> end of its entries
  const int64_t* cgM;     // (t >= 1) surviving group -> its upward message M
  const int2* ccs;        // surviving entry -> (row count, first position in perm)
  const int2* clr;        // (t >= 1) surviving parent entry -> [first, end) of t's entries
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
};


}  // namespace gjk
