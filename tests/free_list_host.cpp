// Host build of the request server's free list (free_list.hpp) for its
// tests: a C interface over one FreeList.
#include "../paper_1809_09851_amd/csrc/free_list.hpp"

static fdbb::FreeList g_list;

extern "C" {
void fl_reset(size_t bytes) { g_list.reset(bytes); }
size_t fl_alloc(size_t bytes) { return g_list.alloc(bytes); }
void fl_release(size_t off, size_t bytes) { g_list.release(off, bytes); }
size_t fl_used(void) { return g_list.used(); }
size_t fl_size(void) { return g_list.size(); }
size_t fl_free_blocks(void) { return g_list.free_blocks(); }
size_t fl_largest_free(void) { return g_list.largest_free(); }
}
