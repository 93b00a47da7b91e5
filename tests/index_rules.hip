// index_rules.hip -- test harness (not part of the library): exports the
// host instantiations of the index rules the kernels use (nyx_types.h), so
// the CPU tests check the compiled functions themselves against brute force.
#include <hip/hip_runtime.h>

#include "nyx_types.h"

extern "C" {

void rules_tiles_for(uint32_t n, uint32_t rows, uint32_t width, uint32_t split_vox, uint32_t tile_vox,
                     uint32_t *row_blocks, uint32_t *col_blocks) {
    const nyx::Tiling t = nyx::tiles_for(n, rows, width, split_vox, tile_vox);
    *row_blocks = t.row_blocks;
    *col_blocks = t.col_blocks;
}

void rules_tile_bounds(uint32_t rows, uint32_t width, uint32_t n_tiles, uint32_t tcols, uint32_t tile,
                       uint32_t *out4) {
    nyx::tile_bounds(rows, width, n_tiles, tcols, tile, out4, out4 + 1, out4 + 2, out4 + 3);
}

uint32_t rules_size_class(uint32_t vox) { return nyx::size_class(vox); }

uint32_t rules_ticket_chunk(int cl) { return nyx::ticket_chunk(cl); }

int rules_classes(void) { return nyx::kClasses; }

uint32_t rules_ticket_offsets(const uint32_t *entries, uint32_t *first) { return nyx::ticket_offsets(entries, first); }

void rules_ticket_range(uint32_t t, const uint32_t *entries, const uint32_t *first, int32_t *cl, uint32_t *e0,
                        uint32_t *e1) {
    int c = 0;
    nyx::ticket_range(t, entries, first, &c, e0, e1);
    *cl = c;
}

uint32_t rules_label_entry(const uint32_t *dict, uint32_t dict_n, uint32_t max_label, uint32_t l) {
    return nyx::label_entry(dict, dict_n, max_label, l);
}

void rules_fbn_levels(const uint32_t *I, uint32_t n, uint32_t vmin, uint32_t vmax, uint32_t ng, uint32_t *out) {
    const double r = nyx::fbn_rcp_up(vmax > vmin ? vmax - vmin : 1u);
    for (uint32_t k = 0; k < n; ++k) out[k] = nyx::fbn_level_rd(I[k], vmin, r, ng);
}

}  // extern "C"
