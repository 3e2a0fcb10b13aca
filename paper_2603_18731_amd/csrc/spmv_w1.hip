// Matrix-free SpMV kernels for keys of 1 padded word.
#define QSD_SPMV_WP 1
#include "spmv_impl.h"
