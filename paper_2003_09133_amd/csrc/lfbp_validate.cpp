// Host-only argument checks of the C ABI (no HIP calls, no HIP headers).
#include "lfbp_validate.h"

#include <algorithm>
#include <initializer_list>

namespace lfbp {

namespace {
constexpr uint64_t LIM31 = uint64_t(1) << 31;
constexpr uint64_t LIM62 = uint64_t(1) << 62;

// a*b, saturating at 2^63 (enough to test against the limits used here).
uint64_t mul_sat(uint64_t a, uint64_t b)
{
    const uint64_t cap = uint64_t(1) << 63;
    if (a != 0 && b > cap / a) return cap;
    return a * b;
}
}  // namespace

int dtype_size(lfbp_dtype dt)
{
    switch (dt) {
        case LFBP_F32: return 4;
        case LFBP_F16: return 2;
        default: return 0;
    }
}

uint64_t shape_elems(const lfbp_shape& s)
{
    uint64_t e = 1;
    for (int64_t v : {s.ns, s.nt, s.nx, s.ny, s.nz}) e = mul_sat(e, v > 0 ? uint64_t(v) : 0);
    return e;
}

lfbp_status check_shape(const lfbp_shape& s, int esize)
{
    if (s.ns < 1 || s.nt < 1 || s.nx < 1 || s.ny < 1 || s.nz < 1) return LFBP_ESHAPE;
    // Odd cell sides (Sec. 4); odd patch sides so that the reflection of
    // Eqs. 8-9 maps 1..ns onto itself and the patch has a centre pixel.
    if (s.ns % 2 == 0 || s.nt % 2 == 0 || s.nx % 2 == 0 || s.ny % 2 == 0) return LFBP_ESHAPE;
    const uint64_t rows = mul_sat(mul_sat(uint64_t(s.ns), uint64_t(s.nt)), uint64_t(s.nx));
    const uint64_t block = mul_sat(mul_sat(uint64_t(s.nx), uint64_t(s.ny)), uint64_t(s.nz));
    if (rows >= LIM31 || block >= LIM31) return LFBP_ESHAPE;
    if (mul_sat(shape_elems(s), uint64_t(esize > 0 ? esize : 1)) >= LIM62) return LFBP_ESHAPE;
    return LFBP_OK;
}

bool ranges_overlap(const void* a, uint64_t na, const void* b, uint64_t nb)
{
    const uint64_t pa = reinterpret_cast<uint64_t>(a), pb = reinterpret_cast<uint64_t>(b);
    return pa < pb + nb && pb < pa + na;
}

lfbp_status check_gather(const void* H, const void* Ht, const lfbp_shape& s, lfbp_dtype dt)
{
    if (!H || !Ht) return LFBP_EINVAL;
    const int es = dtype_size(dt);
    if (es == 0) return LFBP_EDTYPE;
    const lfbp_status st = check_shape(s, es);
    if (st != LFBP_OK) return st;
    if (reinterpret_cast<uint64_t>(H) % es || reinterpret_cast<uint64_t>(Ht) % es) return LFBP_EALIGN;
    const uint64_t bytes = shape_elems(s) * uint64_t(es);
    if (ranges_overlap(H, bytes, Ht, bytes)) return LFBP_EALIAS;
    return LFBP_OK;
}

lfbp_status check_config(const lfbp_gather_config* c)
{
    if (!c) return LFBP_OK;
    if (c->variant < 0 || c->variant > LFBP_GATHER_WIDE) return LFBP_EINVAL;
    if (c->block_threads != 0 && (c->block_threads < 64 || c->block_threads > 512 || c->block_threads % 64))
        return LFBP_EINVAL;
    if (c->rows_in_flight != 0 && c->rows_in_flight != 1 && c->rows_in_flight != 2) return LFBP_EINVAL;
    if (c->tile_bytes < 0 || c->tile_bytes > 65536) return LFBP_EINVAL;
    if (c->vec_per_thread != 0 && c->vec_per_thread != 2 && c->vec_per_thread != 4 && c->vec_per_thread != 8)
        return LFBP_EINVAL;
    if (c->nontemporal < 0 || c->nontemporal > 2) return LFBP_EINVAL;
    if (c->persistent < 0 || c->persistent > 2) return LFBP_EINVAL;
    if (c->grid < 0) return LFBP_EINVAL;
    if (c->waves_per_eu < 0 || c->waves_per_eu > 8) return LFBP_EINVAL;
    if (c->schedule < 0 || c->schedule > 2) return LFBP_EINVAL;
    return LFBP_OK;
}

lfbp_status check_project_shape(const lfbp_shape& s, int64_t R, int64_t C, unsigned ops)
{
    if (R < 1 || C < 1) return LFBP_EINVAL;
    const lfbp_status st = check_shape(s, 4);
    if (st != LFBP_OK) return st;
    if (mul_sat(mul_sat(uint64_t(R), uint64_t(C)), uint64_t(s.nz)) >= LIM31) return LFBP_ESHAPE;
    // Sizes of the projector's operand records (24 floats per stage of 22
    // reduction indices): stage counts, record indices per stage and the
    // workspace must stay inside the kernels' 32-bit grid and index ranges.
    const uint64_t Kr = uint64_t(s.ns + s.nx - 1), Kc = uint64_t(s.nt + s.ny - 1);
    const uint64_t pairs = mul_sat(Kr, Kc);
    if (mul_sat(pairs, uint64_t(s.nz)) >= LIM31) return LFBP_ESHAPE;
    // A record block (96 bytes per record) is addressed with 32-bit offsets:
    // columns (nx*ny*nz, padded), lenslets (padded) and the lenslet grid of g
    // with its zero border must each stay below 2^31 bytes of records.
    // (backward: nx*ny*nz columns; forward: nx*ny classes in boxes, at most
    // twice that many columns)
    const uint64_t classes = mul_sat(uint64_t(s.nx), uint64_t(s.ny));
    const uint64_t cols = std::max(mul_sat(classes, uint64_t(s.nz)), mul_sat(classes, 2)) + 512;
    const uint64_t hs = uint64_t(s.ns - 1) / 2, ht = uint64_t(s.nt - 1) / 2;
    const uint64_t Lr = uint64_t((R + s.nx - 1) / s.nx), Lc = uint64_t((C + s.ny - 1) / s.ny);
    const uint64_t grid = mul_sat(Lr + 2 * ((hs + s.nx - 1) / s.nx), Lc + 2 * ((ht + s.ny - 1) / s.ny));
    const uint64_t lenslets = mul_sat(Lr, Lc) + 64;
    if (mul_sat(cols, 96) >= LIM31 || mul_sat(lenslets, 96) >= LIM31 || mul_sat(grid, 96) >= LIM31 ||
        mul_sat(pairs + 64, 96) >= LIM31)
        return LFBP_ESHAPE;
    if (mul_sat(mul_sat(mul_sat(pairs, uint64_t(s.nz)), cols + lenslets + grid), 96) >= LIM62) return LFBP_ESHAPE;
    // Every launch must count its work-items (256 per workgroup) in 32 bits
    // along each grid dimension: fewer than 2^24 workgroups along x.  The
    // largest x extents: forward, the B-record stages (Kr*Kc*ceil(nz/22)),
    // the g-record grid (classes times depth chunks), the depth transpose of
    // g (R*C/32) and the GEMM (row tiles of 64 lenslets times column tiles of
    // 256 class-box columns; the split count keeps it at most max(tiles,
    // 512)); backward, the GEMM over lenslets and nx*ny*nz columns; gradient,
    // the GEMM over Kr*Kc rows and nx*ny*nz columns.  Stage counts of 22
    // pairs or lenslets stay below 2^24 by the record limits above.
    const uint64_t lim24 = uint64_t(1) << 24;
    const uint64_t nzc = (uint64_t(s.nz) + 21) / 22;
    const uint64_t fwd_cols = mul_sat(classes, 2) + 256, bwd_cols = mul_sat(classes, uint64_t(s.nz));
    auto tiles = [](uint64_t m, uint64_t n) { return mul_sat((m + 63) / 64, (n + 255) / 256); };
    if ((ops & kProjFwd) &&
        (mul_sat(pairs, nzc) >= lim24 || mul_sat(classes, nzc) >= lim24 ||
         (mul_sat(uint64_t(R), uint64_t(C)) + 31) / 32 >= lim24 || tiles(mul_sat(Lr, Lc), fwd_cols) >= lim24))
        return LFBP_ESHAPE;
    if ((ops & kProjBwd) && tiles(mul_sat(Lr, Lc), bwd_cols) >= lim24) return LFBP_ESHAPE;
    if ((ops & kProjGrad) && tiles(pairs, bwd_cols) >= lim24) return LFBP_ESHAPE;
    return LFBP_OK;
}

lfbp_status check_project(const float* psf, const lfbp_shape& s, const float* in2, int64_t R, int64_t C,
                          const float* out, bool forward)
{
    if (!psf || !in2 || !out) return LFBP_EINVAL;
    const lfbp_status st = check_project_shape(s, R, C, forward ? kProjFwd : kProjBwd);
    if (st != LFBP_OK) return st;
    const int64_t image = R * C, volume = image * s.nz;
    const int64_t in2_elems = forward ? volume : image, out_elems = forward ? image : volume;
    const uintptr_t a = reinterpret_cast<uintptr_t>(psf), b = reinterpret_cast<uintptr_t>(in2),
                    c = reinterpret_cast<uintptr_t>(out);
    if (a % 4 || b % 4 || c % 4) return LFBP_EALIGN;
    const uint64_t ob = uint64_t(out_elems) * 4;
    if (ranges_overlap(out, ob, psf, shape_elems(s) * 4) || ranges_overlap(out, ob, in2, uint64_t(in2_elems) * 4))
        return LFBP_EALIAS;
    return LFBP_OK;
}

lfbp_status check_rl(const float* H, const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C,
                     const float* g, const float* norm, const float* g_out)
{
    if (!H || !Ht || !f || !g || !norm || !g_out) return LFBP_EINVAL;
    const lfbp_status st = check_project_shape(s, R, C, kProjFwd | kProjBwd);
    if (st != LFBP_OK) return st;
    for (const float* p : {H, Ht, f, g, norm, g_out})
        if (reinterpret_cast<uintptr_t>(p) % 4) return LFBP_EALIGN;
    const uint64_t psf = shape_elems(s) * 4, img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(s.nz);
    if (ranges_overlap(g_out, vol, H, psf) || ranges_overlap(g_out, vol, Ht, psf) ||
        ranges_overlap(g_out, vol, f, img) || ranges_overlap(g_out, vol, norm, vol))
        return LFBP_EALIAS;
    if (g_out != g && ranges_overlap(g_out, vol, g, vol)) return LFBP_EALIAS;   // in place, or apart
    return LFBP_OK;
}

lfbp_status check_grad_psf(const float* w, const float* g, const lfbp_shape& s, int64_t R, int64_t C,
                           const float* dH)
{
    if (!w || !g || !dH) return LFBP_EINVAL;
    const lfbp_status st = check_project_shape(s, R, C, kProjGrad);
    if (st != LFBP_OK) return st;
    for (const float* p : {w, g, dH})
        if (reinterpret_cast<uintptr_t>(p) % 4) return LFBP_EALIGN;
    const uint64_t psf = shape_elems(s) * 4, img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(s.nz);
    if (ranges_overlap(dH, psf, w, img) || ranges_overlap(dH, psf, g, vol)) return LFBP_EALIAS;
    return LFBP_OK;
}

}  // namespace lfbp
