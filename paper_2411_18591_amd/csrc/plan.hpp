// Plan table: per (dtype, padded ly, padded lx) launch schedule chosen by the
// autotuner (column-pass configuration, chunk size, fields per row-pass
// workgroup), with a strict text
// file format for persisting it.  Host code only.
#pragma once

#include <string>

namespace toprop {

struct PlanEntry {
  int col_variant;  // ColCfg variant of the column pass
  int chunk_mb;     // budget of padded intermediate per chunk [MiB]
  double us;        // measured time of the tuned forward propagation [us]
  int row_fpb = 0;  // fields per row-pass workgroup (0: chosen from the device's occupancy)
};

// dtype: 0 = complex64, 1 = complex128.
bool plan_lookup(int dtype, int ly, int lx, PlanEntry* e);
void plan_store(int dtype, int ly, int lx, const PlanEntry& e);
void plan_clear();
int plan_count();

// Returns 0 on success.  A file that fails any check is rejected as a whole
// (the table is left unchanged) with the reason in *err.
int plan_load_file(const char* path, std::string* err);
int plan_save_file(const char* path, std::string* err);

// Validity of one entry (also used by the C entry points).
bool plan_entry_valid(int dtype, int ly, int lx, const PlanEntry& e, std::string* err);

// The cache file named by TOPROP_PLAN_CACHE (empty if unset); loaded into
// the table once, on first use of the table.  A corrupted cache is ignored
// and rewritten by the next autotune.
const std::string& plan_env_path();

constexpr int kPlanMaxChunkMb = 65536;
constexpr int kPlanMaxRowFpb = 8;

}  // namespace toprop
