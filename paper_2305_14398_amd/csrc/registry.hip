// Operation data provider (Section 5.2.2): custom unitaries registered by
// name, then applied to a contiguous range of qubits.  Entries are immutable
// and never freed, so the host and device copies handed out stay valid for
// the life of the process.
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"

namespace qsim {
namespace {

struct CustomOp {
    std::string name;
    int m = 0;
    std::vector<double> host;          // 2 * 4^m doubles, row-major (re, im)
    std::map<int, double*> device64;   // device -> float64 copy
};

std::mutex g_mu;
std::vector<std::unique_ptr<CustomOp>> g_ops;  // id = index + 1

hipError_t upload(CustomOp& op, int dev, double** out) {
    auto it = op.device64.find(dev);
    if (it != op.device64.end()) {
        *out = it->second;
        return hipSuccess;
    }
    DeviceGuard g(dev);
    if (g.err != hipSuccess) return g.err;
    double* p = nullptr;
    const size_t bytes = op.host.size() * sizeof(double);
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) e = hipMemcpy(p, op.host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p) (void)hipFree(p);
        return e;
    }
    op.device64[dev] = p;
    *out = p;
    return hipSuccess;
}

}  // namespace

int custom_qubits(int32_t id) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (id < 1 || id > (int32_t)g_ops.size()) return 0;
    return g_ops[id - 1]->m;
}

const double* custom_host(int32_t id) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (id < 1 || id > (int32_t)g_ops.size()) return nullptr;
    return g_ops[id - 1]->host.data();
}

qsim_status custom_device(int32_t id, int dev, const double** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (id < 1 || id > (int32_t)g_ops.size()) return fail(QSIM_E_INVALID, "custom operation %d is not registered", id);
    double* p = nullptr;
    hipError_t e = upload(*g_ops[id - 1], dev, &p);
    if (e != hipSuccess) return device_fail("custom operation upload", e);
    *out = p;
    return QSIM_OK;
}

}  // namespace qsim

using namespace qsim;

extern "C" {

qsim_status qsim_register_unitary(const char* name, int n_qubits, const double* matrix, int32_t* id_out) {
    if (name == nullptr || name[0] == '\0') return fail(QSIM_E_INVALID, "name is NULL or empty");
    if (matrix == nullptr || id_out == nullptr) return fail(QSIM_E_INVALID, "matrix or id_out is NULL");
    if (n_qubits < 1 || n_qubits > QSIM_CUSTOM_MAX_QUBITS)
        return fail(QSIM_E_RANGE, "custom operation of %d qubits outside 1..%d", n_qubits, QSIM_CUSTOM_MAX_QUBITS);
    const int D = 1 << n_qubits;
    for (int i = 0; i < 2 * D * D; ++i)
        if (!std::isfinite(matrix[i])) return fail(QSIM_E_INVALID, "custom operation '%s': entry is not finite", name);
    // The registered data must be unitary: M^H M = I (Section 2.3).
    double worst = 0.0;
    for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b) {
            double re = 0.0, im = 0.0;
            for (int r = 0; r < D; ++r) {
                const double ar = matrix[2 * (r * D + a)], ai = matrix[2 * (r * D + a) + 1];
                const double br = matrix[2 * (r * D + b)], bi = matrix[2 * (r * D + b) + 1];
                re += ar * br + ai * bi;  // conj(M[r][a]) * M[r][b]
                im += ar * bi - ai * br;
            }
            if (a == b) re -= 1.0;
            worst = std::fmax(worst, std::hypot(re, im));
        }
    if (worst > 1e-9)
        return fail(QSIM_E_INVALID, "custom operation '%s' is not unitary (max |M^H M - I| = %.3g)", name, worst);

    std::unique_ptr<CustomOp> op(new CustomOp());
    op->name = name;
    op->m = n_qubits;
    op->host.assign(matrix, matrix + 2 * D * D);
    int32_t id = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& o : g_ops)
            if (o->name == op->name) return fail(QSIM_E_INVALID, "custom operation '%s' is already registered", name);
        if ((int)g_ops.size() >= QSIM_CUSTOM_MAX_OPS)
            return fail(QSIM_E_RANGE, "the registry holds %d operations already", QSIM_CUSTOM_MAX_OPS);
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess) count = 0;
        for (int d = 0; d < count; ++d) {
            double* p = nullptr;
            hipError_t e = upload(*op, d, &p);
            if (e != hipSuccess) {
                for (auto& kv : op->device64) {
                    DeviceGuard g(kv.first);
                    (void)hipFree(kv.second);
                }
                return device_fail("custom operation upload", e);
            }
        }
        g_ops.push_back(std::move(op));
        id = (int32_t)g_ops.size();
    }
    *id_out = id;
    return ok();
}

qsim_status qsim_find_unitary(const char* name, int32_t* id_out, int* n_qubits_out) {
    if (name == nullptr) return fail(QSIM_E_INVALID, "name is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = 0; i < g_ops.size(); ++i)
        if (g_ops[i]->name == name) {
            if (id_out) *id_out = (int32_t)(i + 1);
            if (n_qubits_out) *n_qubits_out = g_ops[i]->m;
            return ok();
        }
    return fail(QSIM_E_UNKNOWN_ID, "no custom operation named '%s'", name);
}

}  // extern "C"
