// CKKS bootstrapping of sparsely packed ciphertexts (device program).
#pragma once
#include <stdint.h>

#include <vector>

#include "context.h"

namespace csrmf {

struct BootCfg {
    int n = 0;          // slots of the sparse packing (power of two, 1..N/4)
    int r = 0;          // squarings of the exponential
    int d = 0;          // degree of exp's Taylor series (1..18)
    int pre_bits = 0;   // the level-0 input is multiplied by 2^pre_bits
    bool arcsine = false;   // add the cubic term of arcsin after EvalMod (2 more levels)
};

// Levels one bootstrap consumes: 2 + ceil(log2 d) + 1 + r (+ 2 with the arcsine
// term) + 1.
int boot_levels(const BootCfg& cfg);
// Rotation steps whose keys a bootstrap needs (besides relinearisation and
// conjugation), ascending.
std::vector<int32_t> boot_rotation_steps(uint64_t N, int n);
// Throws Error(CSRMF_E_INVAL) unless cfg is usable on the context's chain.
void boot_check(const Context* c, const BootCfg& cfg);
// Bootstrap in[i] (equal scales, any level, slots n-periodic) into out[i] at
// level L - boot_levels(cfg), scale about 2^log2_scale.
void bootstrap(Context* c, const BootCfg& cfg, const std::vector<Ct*>& in, std::vector<Ct>& out);

}  // namespace csrmf
