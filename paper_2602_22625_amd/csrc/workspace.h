// Growth of the context's device workspace buffers: host logic only, with no HIP types, so the
// same code is exercised by a CPU test against a simulated allocator.
//
// A buffer only grows. Growing it releases the old memory and acquires a larger block; the old
// contents are not kept. Two rules make this safe:
//   - the device is quiesced first (every queued kernel on every stream has finished), so no
//     kernel can still touch the old block, whichever stream it was queued on;
//   - a buffer that must read as zero (tile counters) is cleared whenever a new block was
//     acquired, whatever its address. An allocator may well return the base address of the
//     block just released; the new block's tail past the old capacity then holds whatever the
//     process last stored at those addresses, not zeros.
#pragma once

#include <stddef.h>

namespace dbmp {

struct Buf {
    void *p = nullptr;
    size_t cap = 0;  // bytes
};

// Ops supplies the device operations (each returns 0 on success, else an error code):
//   int quiesce();                        wait until no queued work can touch any buffer
//   void release(void *p);                give a block back
//   int acquire(void **p, size_t bytes);  get a block of at least `bytes`
//   int clear(void *p, size_t bytes);     zero-fill, complete on return
// Returns 0 (buffer large enough, or grown; *grown tells which) or the failing operation's code
// (then the buffer is empty: p == nullptr, cap == 0).
template <class Ops>
int grow_buffer(Buf &b, size_t bytes, bool must_be_zero, Ops &ops, bool *grown)
{
    *grown = false;
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return 0;
    int rc = ops.quiesce();
    if (rc) return rc;
    if (b.p) ops.release(b.p);
    b.p = nullptr;
    b.cap = 0;
    const size_t want = bytes + bytes / 4;  // headroom: a slowly growing workload regrows rarely
    void *p = nullptr;
    rc = ops.acquire(&p, want);
    if (rc) return rc;
    if (must_be_zero) {
        rc = ops.clear(p, want);
        if (rc) {
            ops.release(p);
            return rc;
        }
    }
    b.p = p;
    b.cap = want;
    *grown = true;
    return 0;
}

// Whether the raster kernels can address a padded atlas of B bitmaps of (Hb + 2) x (Wb + 2)
// texels of `esz` bytes: a texel is reached by a 32-bit unsigned byte offset from the atlas
// base, and a bitmap's first texel by an int element offset.
// Elements of the padded atlas: B bitmaps of (Hb + 2) x (Wb + 2) (a one-texel zero border),
// then two zero rows of Wb + 2 texels, which hold an all-zero bilinear cell (zero_cell).
inline long long padded_atlas_elems(long long B, long long Hb, long long Wb)
{
    return B * (Hb + 2) * (Wb + 2) + 2 * (Wb + 2);
}

// Element offset of that all-zero cell: a lane outside a primitive's support samples it, so its
// M and derivatives are exactly zero whatever its weights.
inline long long zero_cell(long long B, long long Hb, long long Wb)
{
    return B * (Hb + 2) * (Wb + 2);
}

inline bool atlas_addressable(long long B, long long Hb, long long Wb, long long esz)
{
    if (B < 1 || Hb < 2 || Wb < 2 || (esz != 2 && esz != 4)) return false;
    const long long elems = padded_atlas_elems(B, Hb, Wb);
    return elems < 2147483647LL && elems * esz < 4294967296LL;
}

}  // namespace dbmp
