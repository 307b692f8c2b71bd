// Batched and serving entry points of libpv3d (placeholders until the
// persistent kernel lands; they report that the form is unavailable).
#include "pv3d_runtime.h"

using namespace pv3d;

namespace pv3d {
bool Ctx::scene_in_use(uint64_t) { return false; }
bool Ctx::gen_in_use(uint64_t) { return false; }
void Ctx::release_batched() {}
}  // namespace pv3d

void pv3d_server_stop(pv3d_ctx*) {}

extern "C" {
pv3d_status pv3d_evaluate_batched(pv3d_ctx* ctx, const pv3d_job* jobs, int64_t n_jobs, void* hip_stream) {
    (void)ctx; (void)jobs; (void)n_jobs; (void)hip_stream;
    return fail(PV3D_ERANGE, "batched evaluation is not available in this build");
}
pv3d_status pv3d_submit(pv3d_ctx* ctx, const pv3d_job* job, uint64_t* ticket) {
    (void)ctx; (void)job; (void)ticket;
    return fail(PV3D_ERANGE, "serving is not available in this build");
}
pv3d_status pv3d_poll(pv3d_ctx* ctx, uint64_t ticket, int32_t* done) {
    (void)ctx; (void)ticket; (void)done;
    return fail(PV3D_ENOENT, "unknown ticket");
}
pv3d_status pv3d_wait(pv3d_ctx* ctx, uint64_t ticket) {
    (void)ctx; (void)ticket;
    return fail(PV3D_ENOENT, "unknown ticket");
}
pv3d_status pv3d_cancel(pv3d_ctx* ctx, uint64_t ticket) {
    (void)ctx; (void)ticket;
    return fail(PV3D_ENOENT, "unknown ticket");
}
}
