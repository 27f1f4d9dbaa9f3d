// Block preconditioner of Sec. 2.3 (eqs. (4)-(5), Fig. 3) -- placeholder
// until the padded-domain operator lands.
#include "ctx.h"

namespace mspcg {

int domains_setup(mspcg_ctx*, const mspcg_blocking&, int, hipStream_t) {
    return MSPCG_EUNSUPPORTED;
}

template <class S>
int precond_apply(mspcg_ctx*, int, CField<F64>, Field<F64>, hipStream_t, int*) {
    return MSPCG_EUNSUPPORTED;
}

template <class S>
int kblock_apply(mspcg_ctx*, CField<F64>, Field<F64>, hipStream_t) {
    return MSPCG_EUNSUPPORTED;
}

template int precond_apply<F64>(mspcg_ctx*, int, CField<F64>, Field<F64>, hipStream_t, int*);
template int precond_apply<F32>(mspcg_ctx*, int, CField<F64>, Field<F64>, hipStream_t, int*);
template int precond_apply<F16>(mspcg_ctx*, int, CField<F64>, Field<F64>, hipStream_t, int*);
template int kblock_apply<F64>(mspcg_ctx*, CField<F64>, Field<F64>, hipStream_t);
template int kblock_apply<F32>(mspcg_ctx*, CField<F64>, Field<F64>, hipStream_t);
template int kblock_apply<F16>(mspcg_ctx*, CField<F64>, Field<F64>, hipStream_t);

}  // namespace mspcg
