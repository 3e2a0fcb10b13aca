// Matrix-free SpMV kernels for keys of 2 padded words.
#define QSD_SPMV_WP 2
#include "spmv_impl.h"
