// lengths.hpp -- transform lengths instantiated by the kernels:
// N = 2^a or 3*2^a.  x uses M = nx/2 <= 1024; y and periodic z use N <= 2048.
#pragma once

#define PK_X_LENGTHS(X)                                                                        \
    X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192)    \
    X(256) X(384) X(512) X(768) X(1024)
#define PK_LENGTHS(X) PK_X_LENGTHS(X) X(1536) X(2048)

#define PK_CAT2(a, b) a##_##b
#define PK_CAT(a, b) PK_CAT2(a, b)
#ifdef PK_TAG
#define PK_SUFFIX(name) PK_CAT(name, PK_TAG)
// Kernels of a precision-templated source live in their own namespace: the
// source is compiled once per precision and the kernel templates are not
// parameterised on the real type, so without it the FP32 and FP64 objects
// would define identically-named kernels and the link would keep only one.
#define PK_NS PK_CAT(prec, PK_TAG)
#endif
