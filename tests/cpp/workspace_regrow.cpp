// Host-logic checks of the context workspace (paper_2602_22625_amd/csrc/workspace.h), run on the
// CPU against a simulated device allocator that behaves like a recycling one: a released block's
// base address is handed out again when the next request fits there, and recycled memory holds
// what was last stored in it (here 0xAB bytes), never zeros.
#include "workspace.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

namespace {

struct RecyclingOps {
    unsigned char *arena = nullptr;  // one region; every block starts at its base
    size_t arena_bytes = 0;
    bool live = false;
    std::vector<std::string> log;  // the order of the operations
    int quiesce()
    {
        log.push_back("quiesce");
        return 0;
    }
    void release(void *p)
    {
        log.push_back("release");
        if (p == arena) live = false;
    }
    int acquire(void **p, size_t bytes)
    {
        log.push_back("acquire");
        if (live || bytes > arena_bytes) return -2;
        // the block is the arena's base again; its bytes are whatever was stored there last
        live = true;
        *p = arena;
        return 0;
    }
    int clear(void *p, size_t bytes)
    {
        log.push_back("clear");
        memset(p, 0, bytes);
        return 0;
    }
};

int failures = 0;
#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #cond);                \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

}  // namespace

int main()
{
    using dbmp::Buf;
    using dbmp::grow_buffer;
    RecyclingOps ops;
    ops.arena_bytes = 1 << 20;
    ops.arena = (unsigned char *)malloc(ops.arena_bytes);
    memset(ops.arena, 0xAB, ops.arena_bytes);  // stale contents of recycled memory

    // tile counters for 4,096 tiles (a 512 x 512 canvas at 8 x 8 tiles), then 16,384 tiles (a
    // 2048 x 2048 canvas at 16 x 16): the second block has the first one's base address
    Buf counts;
    bool grown = false;
    CHECK(grow_buffer(counts, 4 * 4096, true, ops, &grown) == 0 && grown);
    void *first = counts.p;
    // the forward re-arms every counter it used; the memory past them stays stale
    memset(counts.p, 0, 4 * 4096);
    CHECK(grow_buffer(counts, 4 * 16384, true, ops, &grown) == 0 && grown);
    CHECK(counts.p == first);  // the allocator reused the address
    CHECK(counts.cap >= 4 * 16384);
    const int *c = (const int *)counts.p;
    int nonzero = 0;
    for (size_t i = 0; i < counts.cap / 4; ++i) nonzero += c[i] != 0;
    CHECK(nonzero == 0);  // every counter of the larger canvas starts at zero

    // the device is quiesced before the old block is released, and the clear follows the
    // acquisition
    const std::vector<std::string> want = {"quiesce", "acquire", "clear",  "quiesce",
                                           "release", "acquire", "clear"};
    CHECK(ops.log == want);

    // a request that fits changes nothing
    ops.log.clear();
    CHECK(grow_buffer(counts, 4 * 1000, true, ops, &grown) == 0 && !grown);
    CHECK(ops.log.empty());

    // a buffer that need not be zero is not cleared
    Buf lists;
    RecyclingOps ops2;
    ops2.arena_bytes = 1 << 16;
    ops2.arena = (unsigned char *)malloc(ops2.arena_bytes);
    CHECK(grow_buffer(lists, 1000, false, ops2, &grown) == 0 && grown);
    const std::vector<std::string> want2 = {"quiesce", "acquire"};
    CHECK(ops2.log == want2);

    // an allocation failure leaves an empty buffer
    Buf big;
    CHECK(grow_buffer(big, (size_t)1 << 30, true, ops2, &grown) != 0 && !grown);
    CHECK(big.p == nullptr && big.cap == 0);

    // atlas sizes the kernels can address (32-bit texel byte offsets)
    CHECK(dbmp::atlas_addressable(64, 128, 128, 2));      // the 2048 x 2048 workload's atlas
    CHECK(dbmp::atlas_addressable(16, 64, 64, 4));
    CHECK(!dbmp::atlas_addressable(0, 64, 64, 4));
    CHECK(!dbmp::atlas_addressable(4, 1, 64, 4));
    CHECK(!dbmp::atlas_addressable(1, 64, 64, 8));
    // 2^18 padded bitmaps of 64 x 64 texels: 2^30 texels, 4 GiB in fp32 (not addressable although
    // fewer than 2^31 texels), 2 GiB in bf16
    CHECK(!dbmp::atlas_addressable(262144, 62, 62, 4));
    CHECK(dbmp::atlas_addressable(262144, 62, 62, 2));
    CHECK(dbmp::atlas_addressable(262143, 62, 62, 4));  // one bitmap fewer: 4 GiB - 16 KiB
    CHECK(!dbmp::atlas_addressable(1, 46341, 46341, 2));  // more than 2^31 texels

    free(ops.arena);
    free(ops2.arena);
    if (failures) return 1;
    printf("workspace checks passed\n");
    return 0;
}
