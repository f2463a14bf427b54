// layout_check.cpp -- host-side check of the workspace arithmetic of qed_step and qed_thin
// (built by tests/test_layout.py with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host code; it launches nothing and needs no GPU).
//
// For the workspace shapes of the benchmark's workloads and for edge cases it checks that
// every region of WorkLayout and ThinLayout is 256-byte aligned, inside the workspace and
// disjoint from the others; that qed_work_bytes and qed_thin_work_bytes return the layouts'
// totals; and that the largest index each kernel can form stays inside its region: the
// photon wavefronts' candidate lists for every wavefront count a launch can have, and the
// child arenas' shares, pool chunks, count matrices and chunk chains for every producer
// (the lepton kernel's grids, the exact pair kernel's, the generation kernel's).  The same
// for the cell sort's workspace (SortLayout) and its key geometry, and for the workspaces of
// the thinning per cell and the cap per parent.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "qed_internal.h"

using namespace qedk;

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      ++failures;                             \
      fprintf(stderr, "FAIL %s: ", #cond);    \
      fprintf(stderr, __VA_ARGS__);           \
      fprintf(stderr, "\n");                  \
    }                                         \
  } while (0)

struct Region {
  size_t off, bytes;
  const char* name;
};

static void check_regions(std::vector<Region> r, size_t begin, size_t total, const char* what) {
  std::sort(r.begin(), r.end(), [](const Region& a, const Region& b) { return a.off < b.off; });
  size_t end = begin;
  for (const Region& x : r) {
    CHECK(x.off % 256 == 0, "%s: %s at %zu is not 256-byte aligned", what, x.name, x.off);
    CHECK(x.off >= end, "%s: %s at %zu overlaps the region before it (ends %zu)", what, x.name,
          x.off, end);
    end = x.off + x.bytes;
    CHECK(end <= total, "%s: %s ends at %zu past the workspace (%zu)", what, x.name, end, total);
  }
}

static void check_arena(const WorkLayout& L, int n_inst, long long cap, bool pair, int waves,
                        bool pool, const char* what) {
  const ArenaGeometry g = arena_geometry(cap, waves, pool);
  // shares and pool chunks inside the record columns
  CHECK(g.pool0 + g.nchunks * kArenaChunk <= cap, "%s: records %lld + %lld chunks > cap %lld",
        what, g.pool0, g.nchunks, cap);
  CHECK(g.per_wave >= 0 && g.nchunks >= 0, "%s: negative geometry", what);
  // record indices are formed in 64-bit but stored as 32-bit chunk numbers and counts
  CHECK(cap < (1ll << 31), "%s: %lld records do not fit 32-bit record numbers", what, cap);
  CHECK(g.nchunks < (1ll << 32) - 1, "%s: chunk numbers overflow", what);
  // count matrix [n_inst][waves] in a region of n_inst * kMaxWaves words; first[] and
  // nrec[] of kMaxWaves words; next[] of cap / kArenaChunk + 1 words
  CHECK(waves <= kMaxWaves, "%s: %d producing wavefronts > %d", what, waves, kMaxWaves);
  const size_t mat = sizeof(unsigned int) * (size_t)n_inst * kMaxWaves;
  CHECK((size_t)n_inst * waves * sizeof(unsigned int) <= mat, "%s: count matrix", what);
  const size_t chain = WorkLayout::ChainBytes(cap);
  const size_t need = 256 + ((sizeof(unsigned int) * kMaxWaves + 255) & ~(size_t)255) +
                      sizeof(unsigned int) * (size_t)(g.nchunks > 0 ? g.nchunks : 1);
  CHECK(need <= chain, "%s: chunk chain needs %zu of %zu bytes", what, need, chain);
  // the columns: 7 (pair: 8) doubles, parent, sub and instance, plus the same-step columns
  const size_t col8 = ((size_t)cap * 8 + 255) & ~(size_t)255;
  const size_t col4 = ((size_t)cap * 4 + 255) & ~(size_t)255;
  size_t cols = col8 * (pair ? 8 : 7) + col8 + 2 * col4;
  if (L.same_step) cols += col8 * (1 + 6 + (pair ? 2 : 1));
  CHECK(cols <= WorkLayout::ChildArenaBytes(cap, pair, L.same_step), "%s: columns", what);
}

static void check_work(int n_inst, long long slots, long long arena, bool same_step,
                       const char* what) {
  const WorkLayout L = WorkLayout::make(n_inst, slots, arena, same_step);
  const size_t pub = qed_work_bytes(n_inst, slots, arena, same_step ? 1 : 0);
  CHECK(pub == L.total, "%s: qed_work_bytes %zu vs layout %zu", what, pub, L.total);
  const size_t s = (size_t)(slots > 0 ? slots : 1);
  const size_t part = sizeof(unsigned long long) * kPfCount * kMaxGridBlocks;
  std::vector<Region> r = {
      {L.n0, sizeof(long long) * 3 * (size_t)n_inst, "n0"},
      {L.lep_pref, sizeof(long long) * (2 * (size_t)n_inst + 1), "lep_pref"},
      {L.pho_pref, sizeof(long long) * ((size_t)n_inst + 1), "pho_pref"},
      {L.eb, sizeof(double) * 6 * (size_t)n_inst, "eb"},
      {L.lep_part, part, "lep_part"},
      {L.pho_part, part, "pho_part"},
      {L.ex_part, part, "ex_part"},
      {L.candn, sizeof(unsigned int) * kMaxWaves, "candn"},
      {L.candw, sizeof(unsigned long long) * (s + (size_t)kMaxWaves * kCandSlack), "candw"},
      {L.cand, sizeof(unsigned long long) * s, "cand"}};
  const bool arenas = arena > 0 && n_inst <= kArenaMaxInstances;
  if (arenas) {
    for (int k = 0; k < (same_step ? 2 : 1); ++k) {
      const size_t mat = sizeof(unsigned int) * (size_t)n_inst * kMaxWaves;
      r.push_back({L.ph_cols[k], WorkLayout::ChildArenaBytes(L.ph_cap, false, same_step), "ph_cols"});
      r.push_back({L.ph_cnt[k], mat, "ph_cnt"});
      r.push_back({L.ph_nrec[k], sizeof(unsigned int) * kMaxWaves, "ph_nrec"});
      r.push_back({L.ph_base[k], sizeof(long long) * 2 * (size_t)n_inst, "ph_base"});
      r.push_back({L.ph_chain[k], WorkLayout::ChainBytes(L.ph_cap), "ph_chain"});
      r.push_back({L.pr_cols[k], WorkLayout::ChildArenaBytes(L.pr_cap, true, same_step), "pr_cols"});
      r.push_back({L.pr_cnt[k], mat, "pr_cnt"});
      r.push_back({L.pr_nrec[k], sizeof(unsigned int) * kMaxWaves, "pr_nrec"});
      r.push_back({L.pr_base[k], sizeof(long long) * 2 * (size_t)n_inst, "pr_base"});
      r.push_back({L.pr_chain[k], WorkLayout::ChainBytes(L.pr_cap), "pr_chain"});
    }
    if (same_step) r.push_back({L.gen_part, part, "gen_part"});
  }
  check_regions(r, sizeof(WorkHdr), L.total, what);
  // candidate lists: every photon-kernel wavefront count (grids up to kMaxGridBlocks
  // workgroups of 1..4 wavefronts)
  for (int w = 1; w <= kMaxWaves; w += (w < 64 ? 1 : 61)) {
    const long long per = cand_list_entries(slots, w);
    CHECK((size_t)per * w <= s + (size_t)kMaxWaves * kCandSlack,
          "%s: %d photon wavefronts x %lld entries past the lists", what, w, per);
  }
  // arenas, for every producer: lepton grids of 1..kMaxGridBlocks workgroups of 1..4
  // wavefronts (with and without a pool), the exact pair kernel, the generation kernel
  if (arenas) {
    for (int w = 1; w <= kMaxWaves; w = w < 64 ? w + 1 : w * 2 + 3) {
      check_arena(L, n_inst, L.ph_cap, false, w, false, what);
      check_arena(L, n_inst, L.ph_cap, false, w, true, what);
    }
    check_arena(L, n_inst, L.ph_cap, false, kMaxWaves, true, what);
    check_arena(L, n_inst, L.pr_cap, true, kExactGridBlocks * 4, true, what);
    if (same_step) {
      check_arena(L, n_inst, L.ph_cap, false, kGenGridBlocks * 4, true, what);
      check_arena(L, n_inst, L.pr_cap, true, kGenGridBlocks * 4, true, what);
    }
  }
}

static void check_thin(int n_inst, long long slots, const char* what) {
  const ThinLayout T = ThinLayout::make(n_inst, slots);
  CHECK(qed_thin_work_bytes(n_inst, slots) == T.total, "%s: qed_thin_work_bytes", what);
  CHECK(T.nb >= 1 && T.nb <= kThinBlocks, "%s: %d ranges", what, T.nb);
  const size_t nb = (size_t)n_inst * T.nb;
  std::vector<Region> r = {{T.plan, 64 * (size_t)n_inst, "plan"},
                           {T.part_n, 8 * nb, "part_n"},
                           {T.part_w, 8 * nb, "part_w"},
                           {T.hole_off, 8 * nb, "hole_off"},
                           {T.surv_off, 8 * nb, "surv_off"},
                           {T.holes, 4 * (size_t)(slots > 0 ? slots : 1), "holes"}};
  check_regions(r, 0, T.total, what);
  // the holes of one segment are numbered by 32-bit slot offsets
  CHECK(slots < (1ll << 32), "%s: 32-bit hole list", what);
}

// qed_sort_cells: regions of SortLayout, the public size, and the indices the sort kernels
// form for `slots` slots over n_inst instances (every tile list, count matrix and scan
// chunk the prep kernel can produce), plus the key geometry of a grid.
static void check_sort(int n_inst, long long slots, const char* what) {
  const SortLayout L = SortLayout::make(n_inst, slots);
  CHECK(qed_sort_work_bytes(n_inst, slots) == L.total, "%s: qed_sort_work_bytes", what);
  const size_t cap = (size_t)L.cap;
  const size_t col8 = (cap * 8 + 255) & ~(size_t)255, col4 = (cap * 4 + 255) & ~(size_t)255;
  const size_t chunks = ((size_t)L.tiles_max * 256 + 4095) / 4096;
  std::vector<Region> r = {{L.hdr, sizeof(SortHdr), "hdr"},
                           {L.gpref, 8 * ((size_t)n_inst + 1), "gpref"},
                           {L.tpref, 8 * ((size_t)n_inst + 1), "tpref"},
                           {L.key[0], 4 * cap, "key0"},
                           {L.key[1], 4 * cap, "key1"},
                           {L.val[0], 4 * cap, "val0"},
                           {L.val[1], 4 * cap, "val1"},
                           {L.cnt, 4 * 256 * (size_t)L.tiles_max, "cnt"},
                           {L.sums, 4 * chunks, "sums"},
                           {L.cols, 9 * col8 + 2 * col4, "cols"}};
  check_regions(r, 0, L.total, what);
  // the most tiles: every instance's last tile partial (live counts summing to the slots)
  const long long s = slots > 0 ? slots : 0;
  const long long worst = (n_inst <= s ? (s - n_inst) / kSortTile + n_inst : s);
  CHECK(worst <= L.tiles_max, "%s: %lld tiles > %lld", what, worst, L.tiles_max);
  CHECK(L.tiles_max < (1ll << 31), "%s: tile grid of %lld workgroups", what, L.tiles_max);
  CHECK(chunks < (1ull << 31), "%s: scan grid", what);
  CHECK(s < (1ll << 32), "%s: 32-bit item indices", what);
}

// qed_thin_cells: the sort's regions, then its own; the per-tile group and survivor counts
// share the sort's count array (2 x tiles_max of its 256 x tiles_max words).
static void check_thin_cells(int n_inst, long long slots, const char* what) {
  const ThinCellsLayout L = ThinCellsLayout::make(n_inst, slots);
  CHECK(qed_thin_cells_work_bytes(n_inst, slots) == L.total, "%s: qed_thin_cells_work_bytes",
        what);
  const SortLayout& S = L.sort;
  const size_t cap = (size_t)S.cap;
  std::vector<Region> r = {{S.hdr, sizeof(SortHdr), "hdr"},
                           {S.gpref, 8 * ((size_t)n_inst + 1), "gpref"},
                           {S.tpref, 8 * ((size_t)n_inst + 1), "tpref"},
                           {S.key[0], 4 * cap, "key0"},
                           {S.key[1], 4 * cap, "key1"},
                           {S.val[0], 4 * cap, "val0"},
                           {S.val[1], 4 * cap, "val1"},
                           {S.cnt, 4 * 256 * (size_t)S.tiles_max, "cnt"},
                           {S.sums, 4 * (((size_t)S.tiles_max * 256 + 4095) / 4096), "sums"},
                           {S.cols, 9 * ((cap * 8 + 255) & ~(size_t)255) +
                                        2 * ((cap * 4 + 255) & ~(size_t)255), "cols"},
                           {L.gstart, 4 * (cap + 1), "gstart"},
                           {L.gfac, 8 * cap, "gfac"},
                           {L.gw, 8 * cap, "gw"},
                           {L.gwa, 8 * cap, "gwa"},
                           {L.gkept, 4 * cap, "gkept"},
                           {L.big, 4 * cap, "big"},
                           {L.gpfx, 8 * ((size_t)n_inst + 1), "gpfx"},
                           {L.kpref, 8 * ((size_t)n_inst + 1), "kpref"}};
  check_regions(r, 0, L.total, what);
  CHECK(L.gstart >= S.total, "%s: thinning regions overlap the sort's", what);
  CHECK(2 * (size_t)S.tiles_max <= 256 * (size_t)S.tiles_max, "%s: tile counts", what);
}

// qed_thin_children: the hash tables (2 entries per slot), entry indices, keep flags, the
// column copy, and per (instance, range) partials and offsets; a table entry is a 32-bit
// index below 2 x capacity, so stores of fewer than 2^31 slots.
static void check_thin_children(int n_inst, long long slots, const char* what) {
  const ThinChildrenLayout L = ThinChildrenLayout::make(n_inst, slots);
  CHECK(qed_thin_children_work_bytes(n_inst, slots) == L.total,
        "%s: qed_thin_children_work_bytes", what);
  const size_t n = (size_t)(slots > 0 ? slots : 1);
  const size_t nb = (size_t)n_inst * L.nb;
  std::vector<Region> r = {{L.hdr, 64 * (size_t)n_inst, "hdr"}, {L.part, 64 * nb, "part"},
                           {L.off, 8 * nb, "off"},          {L.tkey, 16 * n, "tkey"},
                           {L.tn, 8 * n, "tn"},             {L.tk, 8 * n, "tk"},
                           {L.tk2, 8 * n, "tk2"},           {L.tmin, 16 * n, "tmin"},
                           {L.ent, 4 * n, "ent"},           {L.keep, n, "keep"},
                           {L.cd, 56 * n, "cd"},            {L.cu, 16 * n, "cu"},
                           {L.cb, 8 * n, "cb"}};
  check_regions(r, 0, L.total, what);
  CHECK(L.nb >= 1 && L.nb <= kThinBlocks, "%s: %d ranges", what, L.nb);
  if (slots < (1ll << 31))
    CHECK((unsigned long long)(2 * n - 1) <= 0xFFFFFFFEull, "%s: entry indices overflow", what);
  // the documented size: 141 bytes per slot, 72 per instance and range, 64 per instance,
  // plus the alignment of 13 regions
  const size_t doc = 141 * n + 72 * nb + 64 * (size_t)n_inst;
  CHECK(L.total >= doc && L.total <= doc + 13 * 256, "%s: %zu bytes against %zu documented",
        what, L.total, doc);
}

static void check_sort_geometry(int nx, int ny, int nz) {
  const int n[3] = {nx, ny, nz};
  const SortGeometry g = sort_geometry(n);
  long long blocks = 1;
  for (int d = 0; d < 3; ++d) {
    CHECK(g.nb[d] == (((long long)n[d] + (1ll << g.shift) - 1) >> g.shift), "nb %d", d);
    CHECK(((long long)(n[d] - 1) >> g.shift) < g.nb[d], "last cell's block %d", d);
    blocks *= g.nb[d];
  }
  CHECK(g.passes >= 1 && g.passes <= kSortMaxPasses, "%d passes", g.passes);
  CHECK(g.dead == (unsigned)((1ull << (8 * g.passes)) - 1), "dead key %u", g.dead);
  // block keys 0 .. blocks - 1 stay below the non-finite key dead - 1
  CHECK(blocks <= (long long)g.dead - 1, "%dx%dx%d: %lld blocks for dead key %u", nx, ny, nz,
        blocks, g.dead);
  if (g.shift > 0) {  // the smallest shift: one less would not fit
    long long b = 1;
    for (int d = 0; d < 3; ++d) b *= ((long long)n[d] + (1ll << (g.shift - 1)) - 1) >> (g.shift - 1);
    CHECK(b > (1ll << 24) - 2, "%dx%dx%d: shift %d is not the smallest", nx, ny, nz, g.shift);
  }
  if (g.passes > 1)  // the fewest passes
    CHECK(blocks > (1ll << (8 * (g.passes - 1))) - 2, "%dx%dx%d: %d passes", nx, ny, nz,
          g.passes);
}

int main() {
  const long long M = 1000000;
  struct W {
    int n;
    long long slots, arena;
    bool ss;
    const char* what;
  } cases[] = {
      {1, 100 * M, 100 * M / 8, false, "rotating cascade, 10^8 photon slots"},
      {1, 100 * M, 100 * M / 32, false, "rotating cascade, arena slots/32"},
      {1, 100 * M, 100 * M / 2, false, "rotating cascade, arena slots/2"},
      {1, 200 * M, 200 * M / 8, false, "standing wave on the 256^3 grid"},
      {64, 200 * M, 200 * M / 8, false, "batched ensemble of 64"},
      {8, 300 * M, 1ll << 27, true, "shower, same-step children"},
      {8, 200 * M, 1ll << 27, true, "avalanche, same-step children"},
      {1, 400000, 50000, false, "parity cascade"},
      {1, 1, 0, false, "one photon slot, no arena"},
      {1, 0, 0, false, "no photon slots"},
      {1024, 1 * M, 100000, true, "1024 instances (the arena limit)"},
      {1025, 1 * M, 100000, false, "1025 instances (no arenas)"},
      {3, 12 * M, (1ll << 31) - 1, false, "largest arena"},
  };
  for (const W& c : cases) check_work(c.n, c.slots, c.arena, c.ss, c.what);
  check_thin(1, 100 * M, "thin, 10^8 slots");
  check_thin(64, 200 * M, "thin, 64 instances");
  check_thin(1, 1, "thin, one slot");
  check_thin(5, 0, "thin, no slots");
  check_thin(1, (1ll << 32) - 1, "thin, largest store");
  check_sort(1, 200 * M, "sort, 2*10^8 photon slots");
  check_sort(1, 25 * M, "sort, 2.5*10^7 lepton slots");
  check_sort(64, 200 * M, "sort, 64 instances");
  check_sort(1024, 1 * M, "sort, 1024 instances");
  check_sort(5, 0, "sort, no slots");
  check_sort(3, 2, "sort, fewer slots than instances");
  check_sort(1, (1ll << 32) - 1, "sort, largest store");
  check_thin_cells(1, 200 * M, "thin cells, 2*10^8 photon slots");
  check_thin_cells(64, 200 * M, "thin cells, 64 instances");
  check_thin_cells(5, 0, "thin cells, no slots");
  check_thin_cells(1, (1ll << 32) - 1, "thin cells, largest store");
  check_thin_children(1, 200 * M, "thin children, 2*10^8 photon slots");
  check_thin_children(64, 200 * M, "thin children, 64 instances");
  check_thin_children(5, 0, "thin children, no slots");
  check_thin_children(3, 2, "thin children, fewer slots than instances");
  check_thin_children(1, (1ll << 31) - 1, "thin children, largest store");
  const int grids[][3] = {{1, 1, 1}, {7, 5, 4}, {40, 40, 40}, {254, 1, 1}, {255, 1, 1},
                          {256, 256, 256}, {300, 300, 300}, {300, 2, 9}, {65534, 1, 1},
                          {65535, 1, 1}, {1 << 20, 1 << 5, 1 << 5}, {2147483647, 1, 1}};
  for (const auto& g : grids) check_sort_geometry(g[0], g[1], g[2]);
  printf("%s: %d failure(s)\n", failures ? "FAIL" : "ok", failures);
  return failures ? 1 : 0;
}
