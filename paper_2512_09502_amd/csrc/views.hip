// Typed views of the prepared network: the connection arrays with their
// first-index array, the image map of one (group, source host), the
// point-to-point send lists and the collective arrays of one group.  Each
// view only gathers the pointers and sizes that snnc_get_array hands out
// (no copy, no device work); snnc_copy_to_host copies one array into caller
// memory.
#include "internal.h"

using namespace snnc;

namespace {

struct ArrayRef {
    const void* p = nullptr;
    uint64_t n = 0;
    int32_t on_host = 0;
};

// The array if the prepared context holds it; `required` arrays raise the
// accessor's status, the others (some exist at certain memory levels only)
// come back empty.
snnc_status fetch(snnc_ctx* c, int32_t id, ArrayRef& a, bool required) {
    a = ArrayRef{};
    snnc_status st = snnc_get_array(c, id, &a.p, &a.n);
    if (st != SNNC_OK) {
        if (required) return st;
        a = ArrayRef{};
        c->last_error.clear();
        return SNNC_OK;
    }
    st = snnc_array_on_host(c, id, &a.on_host);
    return required ? st : SNNC_OK;
}

snnc_status fail(snnc_ctx* c, snnc_status code, const char* msg) {
    c->last_error = msg;
    return code;
}

// rank of group alpha among the groups of the network, or -1
int64_t group_rank(snnc_ctx* c, int32_t alpha, snnc_status* st) {
    ArrayRef g;
    *st = fetch(c, SNNC_GROUPS, g, true);
    if (*st != SNNC_OK || !g.n) return -1;
    std::vector<int32_t> ids(g.n);
    if (g.on_host) {
        memcpy(ids.data(), g.p, g.n * 4);
    } else {
        *st = snnc_copy_array(c, SNNC_GROUPS, ids.data(), g.n * 4);
        if (*st != SNNC_OK) return -1;
    }
    for (uint64_t k = 0; k < g.n; ++k)
        if (ids[k] == alpha) return (int64_t)k;
    return -1;
}

// entry [i] of a uint64/int64 array, wherever it lives
template <class T>
snnc_status read_entry(snnc_ctx* c, int32_t id, const ArrayRef& a, uint64_t i, T* out) {
    if (i >= a.n) return fail(c, SNNC_EINVAL, "index outside the array");
    if (a.on_host) {
        *out = static_cast<const T*>(a.p)[i];
        return SNNC_OK;
    }
    return snnc_copy_range(c, id, i, 1, out);
}

}  // namespace

extern "C" {

snnc_status snnc_get_connections(const snnc_ctx* cc, snnc_conn_view* v) {
    snnc_ctx* c = const_cast<snnc_ctx*>(cc);
    if (!c || !v) return SNNC_EINVAL;
    *v = snnc_conn_view{};
    if (!c->prepared) return fail(c, SNNC_ESTATE, "connections are indexed by snnc_prepare");
    ArrayRef s, t, d, w, rp, f, k;
    snnc_status st;
    if ((st = fetch(c, SNNC_SRC, s, true)) || (st = fetch(c, SNNC_TGT, t, true)) ||
        (st = fetch(c, SNNC_DELAY, d, true)) || (st = fetch(c, SNNC_WEIGHT, w, true)) ||
        (st = fetch(c, SNNC_ROW_PTR, rp, true)) || (st = fetch(c, SNNC_IMG_FIRST, f, false)) ||
        (st = fetch(c, SNNC_IMG_COUNT, k, false)))
        return st;
    v->src = static_cast<const int32_t*>(s.p);
    v->tgt = static_cast<const int32_t*>(t.p);
    v->delay = static_cast<const uint16_t*>(d.p);
    v->weight = static_cast<const float*>(w.p);
    v->row_ptr = static_cast<const uint64_t*>(rp.p);
    v->img_first = static_cast<const uint64_t*>(f.p);
    v->img_count = static_cast<const uint32_t*>(k.p);
    v->n = s.n;
    v->n_rows = rp.n ? rp.n - 1 : 0;
    v->M_local = c->M[c->P_local];
    v->n_images = c->n_img;
    v->img_rows_on_host = (f.n && f.on_host) || (k.n && k.on_host) ? 1 : 0;
    c->last_error.clear();
    return SNNC_OK;
}

snnc_status snnc_get_image_map(const snnc_ctx* cc, int32_t alpha, uint32_t sigma, const int32_t** R, uint64_t* n,
                               int64_t* img_base, const int32_t** L) {
    snnc_ctx* c = const_cast<snnc_ctx*>(cc);
    if (!c || !R || !n || !img_base) return SNNC_EINVAL;
    *R = nullptr;
    *n = 0;
    *img_base = -1;
    if (L) *L = nullptr;
    if (!c->prepared) return fail(c, SNNC_ESTATE, "the image map is built by snnc_prepare");
    if (alpha < -1) return fail(c, SNNC_EINVAL, "group index below -1");
    if (sigma >= c->P) return fail(c, SNNC_EINVAL, "source host out of range");
    ArrayRef off, rv, lv, base;
    snnc_status st;
    if ((st = fetch(c, SNNC_R_OFF, off, true)) || (st = fetch(c, SNNC_R_VAL, rv, true)) ||
        (st = fetch(c, SNNC_L_VAL, lv, true)) || (st = fetch(c, SNNC_IMG_BASE, base, true)))
        return st;
    // map slots: a = alpha + 1 over the map indices the network has
    const uint64_t slot = (uint64_t)(alpha + 1) * c->P + sigma;
    if (slot + 1 >= off.n) {   // a map index beyond the network's: an empty map
        c->last_error.clear();
        return SNNC_OK;
    }
    uint64_t a = 0, b = 0;
    if ((st = read_entry(c, SNNC_R_OFF, off, slot, &a)) || (st = read_entry(c, SNNC_R_OFF, off, slot + 1, &b)) ||
        (st = read_entry(c, SNNC_IMG_BASE, base, slot, img_base)))
        return st;
    *n = b - a;
    if (b > a) {
        *R = static_cast<const int32_t*>(rv.p) + a;
        if (L) *L = static_cast<const int32_t*>(lv.p) + a;
    }
    c->last_error.clear();
    return SNNC_OK;
}

snnc_status snnc_get_p2p_send(const snnc_ctx* cc, snnc_p2p_view* v) {
    snnc_ctx* c = const_cast<snnc_ctx*>(cc);
    if (!c || !v) return SNNC_EINVAL;
    *v = snnc_p2p_view{};
    if (!c->prepared) return fail(c, SNNC_ESTATE, "the send lists are built by snnc_prepare");
    ArrayRef so, sv, tp, tv, pv;
    snnc_status st;
    if ((st = fetch(c, SNNC_S_OFF, so, true)) || (st = fetch(c, SNNC_S_VAL, sv, true)) ||
        (st = fetch(c, SNNC_TP_PTR, tp, true)) || (st = fetch(c, SNNC_T_VAL, tv, true)) ||
        (st = fetch(c, SNNC_P_VAL, pv, true)))
        return st;
    v->s_off = static_cast<const uint64_t*>(so.p);
    v->s_val = static_cast<const int32_t*>(sv.p);
    v->tp_ptr = static_cast<const uint64_t*>(tp.p);
    v->t_val = static_cast<const uint32_t*>(tv.p);
    v->p_val = static_cast<const uint32_t*>(pv.p);
    v->P = c->P;
    v->M_local = c->M[c->P_local];
    v->n_s = sv.n;
    v->n_tp = tv.n;
    c->last_error.clear();
    return SNNC_OK;
}

snnc_status snnc_get_collective(const snnc_ctx* cc, int32_t alpha, snnc_coll_view* v) {
    snnc_ctx* c = const_cast<snnc_ctx*>(cc);
    if (!c || !v) return SNNC_EINVAL;
    *v = snnc_coll_view{};
    if (!c->prepared) return fail(c, SNNC_ESTATE, "the collective arrays are built by snnc_prepare");
    if (alpha < 0) return fail(c, SNNC_EINVAL, "collective groups are numbered from 0");
    snnc_status st;
    const int64_t g = group_rank(c, alpha, &st);
    if (st != SNNC_OK) return st;
    if (g < 0) return fail(c, SNNC_EINVAL, "no collective call of this group");
    ArrayRef ho, hv, iv, gq, gv, qv;
    if ((st = fetch(c, SNNC_H_OFF, ho, true)) || (st = fetch(c, SNNC_H_VAL, hv, true)) ||
        (st = fetch(c, SNNC_I_VAL, iv, true)) || (st = fetch(c, SNNC_GQ_PTR, gq, true)) ||
        (st = fetch(c, SNNC_G_VAL, gv, true)) || (st = fetch(c, SNNC_Q_VAL, qv, true)))
        return st;
    if ((uint64_t)(g + 1) * c->P >= ho.n) return fail(c, SNNC_EDEVICE, "collective offsets shorter than the groups");
    v->alpha = alpha;
    v->rank = (uint32_t)g;
    v->P = c->P;
    v->M_local = c->M[c->P_local];
    v->h_off = static_cast<const uint64_t*>(ho.p) + (uint64_t)g * c->P;
    v->h_val = static_cast<const int32_t*>(hv.p);
    v->i_val = static_cast<const int32_t*>(iv.p);
    v->gq_ptr = static_cast<const uint64_t*>(gq.p);
    v->g_val = static_cast<const int32_t*>(gv.p);
    v->q_val = static_cast<const uint32_t*>(qv.p);
    v->n_h = hv.n;
    v->n_gq = gv.n;
    v->on_host = ho.on_host;
    c->last_error.clear();
    return SNNC_OK;
}

snnc_status snnc_copy_to_host(const snnc_ctx* cc, int32_t id, void* dst, uint64_t bytes) {
    snnc_ctx* c = const_cast<snnc_ctx*>(cc);
    if (!c || (!dst && bytes)) return SNNC_EINVAL;
    return snnc_copy_array(c, id, dst, bytes);
}

}  // extern "C"
