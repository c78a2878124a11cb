// Allocation-free rotation (csrmf_rotate_noalloc): the key switch of
// csrmf_rotate with every temporary in one static device buffer, for callers
// that cannot allocate device memory.
#include <cstring>

#include "context.h"

namespace csrmf {

// ------------------------------------------------------------------ static scratch
// Scratch of csrmf_rotate_noalloc, for callers that cannot allocate device
// memory.  In host code `scratch` names a host-side stand-in, never the
// device buffer: the device address comes from hipGetSymbolAddress, once per
// device, and only that address is passed to kernels.
static __device__ __align__(256) uint64_t scratch[kNoAllocScratchBytes / 8];

uint64_t* noalloc_scratch_for_current_device() {
    static std::mutex mu;
    static std::map<int, uint64_t*> addr;
    int dev = 0;
    CSRMF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* p = nullptr;
    CSRMF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = (uint64_t*)p;
    return (uint64_t*)p;
}

void Context::rotate_noalloc(const Ct& in, uint32_t g, Ct& out) {
    const Key& key = key_for(g);
    if (in.d == out.d) throw Error(CSRMF_E_INVAL, "the output ciphertext must differ from the input");
    const int lvl = in.level;
    const int nl = lvl + 1, nr = n_ext(lvl);
    const int nd = (int)lv[lvl].digits.size();
    // coefficient form of c1, the extended digits, u (both polynomials, all
    // Q u P limbs) and the converted P part of u
    const size_t words = (size_t)N * ((size_t)nl + (size_t)nd * nr + 2 * (size_t)nr + 2 * (size_t)nl);
    if (words * 8 > kNoAllocScratchBytes)
        throw Error(CSRMF_E_INVAL, "rotation at this level needs " + std::to_string(words * 8 >> 20) +
                                       " MiB of scratch; the allocation-free buffer holds " +
                                       std::to_string(kNoAllocScratchBytes >> 20) + " MiB");
    if (!noalloc_scratch) throw Error(CSRMF_E_STATE, "no device scratch on this context");
    uint64_t* coef = noalloc_scratch;
    uint64_t* ext = coef + (size_t)nl * N;
    uint64_t* u = ext + (size_t)nd * nr * N;
    uint64_t* conv = u + 2 * (size_t)nr * N;
    RowMap c1 = map_ct(in.d, nl);
    for (int i = 0; i < nl; ++i) c1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    ks_modup(c1, lvl, 1, ext, coef);
    ++n_key_switches;
    const KsArgs ka = ks_args(ext, c1, lvl, 1, key);
    ks_inner(ka, lvl, 1, g, u);
    out.level = lvl;
    out.scale = in.scale;
    ks_moddown(ka, g, u, lvl, 1, map_ct(out.d, nl), map_ct(in.d, nl), g, false, RowMap(), conv);
}

}  // namespace csrmf

extern "C" int csrmf_rotate_noalloc(csrmf_ctx* cx, uint64_t a, int32_t r, uint64_t out) {
    using namespace csrmf;
    Context* c = reinterpret_cast<Context*>(cx);
    if (!c) {
        last_error() = "null context";
        return CSRMF_E_INVAL;
    }
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    try {
        if (a == out) throw Error(CSRMF_E_INVAL, "the output ciphertext must differ from the input");
        const Ct& src = c->get(a);
        Ct& dst = c->get(out);
        const uint32_t g = c->galois_for_step(r);
        if (g == 1) {
            CSRMF_HIP(hipMemcpyAsync(dst.d, src.d, c->ct_words() * 8, hipMemcpyDeviceToDevice, c->stream));
            dst.level = src.level;
            dst.scale = src.scale;
        } else {
            c->rotate_noalloc(src, g, dst);
        }
        last_error().clear();
        return CSRMF_OK;
    } catch (const Error& e) {
        last_error() = e.what();
        return e.code;
    } catch (const std::exception& e) {
        last_error() = e.what();
        return CSRMF_E_DEVICE;
    }
}
