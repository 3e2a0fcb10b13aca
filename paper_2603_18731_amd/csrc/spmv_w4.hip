// Matrix-free SpMV kernels for keys of 4 padded words.
#define QSD_SPMV_WP 4
#include "spmv_impl.h"
