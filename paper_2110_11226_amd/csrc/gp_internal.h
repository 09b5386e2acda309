// gp_internal.h -- declarations shared by the library's host and device
// translation units (not part of the public ABI).
#pragma once

#include <cstdint>
#include <string>

#include "gp.h"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define GP_HD __host__ __device__ __forceinline__
#else
#define GP_HD inline
#endif

namespace gp {

// Arity of every opcode (Sec. III: functions of arity at most two); -1 for an
// unknown opcode.
GP_HD int arity(uint32_t op) {
    if (op <= GP_OP_CONST) return 0;
    if (op <= GP_OP_DIV || (op >= GP_OP_MAX && op <= GP_OP_ATAN2)) return 2;
    if (op < GP_OP_COUNT) return 1;
    // user functions (Sec. V): the arity is fixed by the opcode, whether or
    // not the function is defined (gp_validate_population checks that)
    if (op >= GP_OP_USER1 && op < GP_OP_USER2) return 1;
    if (op >= GP_OP_USER2 && op < GP_OP_LIMIT) return 2;
    return -1;
}
GP_HD bool is_user_op(uint32_t op) { return op >= GP_OP_USER1 && op < GP_OP_LIMIT; }
// built-in binary functions (the ones with a binary index)
GP_HD bool is_builtin_binary(uint32_t op) { return op < GP_OP_COUNT && arity(op) == 2; }

// User function definitions as the kernels take them (by value, a kernel
// argument): definition u (opcode GP_OP_USER1 + u) is nodes[u][0 .. len[u])
// with constants consts[u][..]; len[u] == 0 when undefined.
constexpr int kUserFns = GP_OP_LIMIT - GP_OP_USER1;
struct UserDefs {
    int32_t len[kUserFns];
    uint32_t nodes[kUserFns][GP_USER_MAX_NODES];
    float consts[kUserFns][GP_USER_MAX_CONSTS];
};

// Index of a binary function among the binary ones (ADD..DIV, MAX..ATAN2 ->
// 0..6) and of a unary one among the unary ones (NEG..TAN, ABS..CBRT -> 0..13).
GP_HD uint32_t binary_index(uint32_t op) { return op <= GP_OP_DIV ? op - GP_OP_ADD : op - GP_OP_MAX + 4u; }
GP_HD uint32_t unary_index(uint32_t op) { return op <= GP_OP_TAN ? op - GP_OP_NEG : op - GP_OP_ABS + 6u; }

// Philox4x32-10 (Salmon et al., SC'11), the counter-based generator of
// Sec. III-B.  One call maps a 128-bit counter and a 64-bit key to four
// 32-bit words through ten rounds of two 32x32->64 multiplies, with the key
// advanced by the golden-ratio Weyl increments between rounds.
struct Philox4 {
    uint32_t v[4];
};

GP_HD Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed) {
    uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t m1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n1 = static_cast<uint32_t>(m1);
        const uint32_t n2 = static_cast<uint32_t>(m0 >> 32) ^ c3 ^ k1;
        const uint32_t n3 = static_cast<uint32_t>(m0);
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// Stream tags of the counter's fourth word.
enum : uint32_t { kStreamTournament = 0, kStreamInit = 1, kStreamMutation = 2, kStreamDonor = 3 };

// floor(word * n / 2^32): a draw in [0, n).
GP_HD uint32_t below(uint32_t word, uint32_t n) {
    return static_cast<uint32_t>((static_cast<uint64_t>(word) * n) >> 32);
}
// (word >> 8) * 2^-24: a float in [0, 1).
GP_HD float unit(uint32_t word) {
    return static_cast<float>(word >> 8) * (1.0f / 16777216.0f);
}

// Thread-local error text behind gp_last_error().
gp_status fail(gp_status st, const std::string& msg);
gp_status ok();

// The process-wide user function registry (gp_register_function): a copy
// of the definitions, and the bit (1 << op) of every defined opcode.
void user_defs(UserDefs* out);
uint32_t user_defined_mask();
// The built-in functions' bits of function_mask, and every bit a mask may
// hold now (built-ins plus defined user functions).
constexpr uint32_t kBuiltinMask = ((1u << GP_OP_COUNT) - 1u) & ~3u;
inline uint32_t allowed_function_mask() { return kBuiltinMask | user_defined_mask(); }

#if defined(__HIPCC__)
// Returns GP_ERR_DEVICE with the runtime's message when a HIP call fails.
#define GP_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(GP_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// Device buffers of the mutation pipeline (gp_mutate.hip): donor lengths,
// constant counts and offsets, offspring plans, lengths and constant
// counts ([n + 1] each), and the donors themselves.
struct MutateWork {
    int64_t *dlen = nullptr, *dnc = nullptr, *doff = nullptr, *dcoff = nullptr, *clen = nullptr, *cnc = nullptr;
    int64_t dlen_cap = 0, dnc_cap = 0, doff_cap = 0, dcoff_cap = 0, clen_cap = 0, cnc_cap = 0;
    int4* plan = nullptr;
    int64_t plan_cap = 0;
    uint32_t* dnodes = nullptr;
    float* dconsts = nullptr;
    int64_t dnodes_cap = 0, dconsts_cap = 0, donor_cap = 0;
};

gp_status mutate_check(const gp_evolve_params* ev, const gp_init_params* in, int32_t n_offspring, const char* who);
gp_status mutate_work_reserve(MutateWork* w, int32_t n_offspring, const gp_init_params& in);
void mutate_work_free(MutateWork* w);
// The generation number is d_gen[0] when d_gen is not NULL, else gen.
gp_status plan_launch(const gp_evolve_params& ev, int32_t n_offspring, uint32_t gen, const uint32_t* d_gen,
                      int32_t* ops, int32_t* first, int32_t* n_tournaments, hipStream_t s);
gp_status mutate_launch(MutateWork& w, const gp_evolve_params& ev, const gp_init_params& in,
                        const gp_population_dev& par, const int32_t* ops, const int32_t* first, const int32_t* winners,
                        int32_t n_winners, int32_t n_offspring, uint32_t gen, const uint32_t* d_gen,
                        const gp_population_out_dev& out, int64_t* info, hipStream_t s);
#endif

}  // namespace gp
