// Device operator functors (common.h) built from the library's device copy of
// an operator, in either precision.
#pragma once

#include "launch.h"

namespace sstep {

template <typename T>
inline OpPoisson7<T> make_poisson(const OpDev &op)
{
    return OpPoisson7<T>{op.g, op.precond ? T(1) / T(6) : T(1)};
}

template <typename T>
inline OpPoisson27<T> make_poisson27(const OpDev &op)
{
    return OpPoisson27<T>{op.g, op.precond ? T(1) / T(26) : T(1)};
}

template <typename T>
struct Ops;
template <>
struct Ops<double> {
    static OpFaces7<double> faces(const OpDev &op) { return {op.g, op.kx, op.ky, op.kz, op.precond}; }
    static OpCsr<double> csr(const OpDev &op) { return {op.rp, op.ci, op.val, op.invd}; }
    static OpEll<double> ell(const OpDev &op) { return {op.ell_col, op.ell_val, op.ell_off, nullptr, op.precond}; }
};
template <>
struct Ops<float> {
    static OpFaces7<float> faces(const OpDev &op) { return {op.g, op.kx32, op.ky32, op.kz32, op.precond}; }
    static OpCsr<float> csr(const OpDev &op) { return {op.rp, op.ci, op.val32, op.invd32}; }
    static OpEll<float> ell(const OpDev &op) { return {op.ell_col, op.ell_val32, op.ell_off, op.invd32, op.precond}; }
};

}  // namespace sstep
