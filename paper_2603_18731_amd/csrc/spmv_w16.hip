// Matrix-free SpMV kernels for keys of 16 padded words.
#define QSD_SPMV_WP 16
#include "spmv_impl.h"
