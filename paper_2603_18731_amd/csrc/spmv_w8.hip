// Matrix-free SpMV kernels for keys of 8 padded words.
#define QSD_SPMV_WP 8
#include "spmv_impl.h"
