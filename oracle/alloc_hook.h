/* Allocation fault injection for the sanitizer check of the oracle (test
 * infrastructure).  Forced into dof_oracle.c with -include by that build
 * only: every malloc / calloc goes through hooks that the check program
 * defines, which can make the n-th allocation fail so that each error path
 * runs once under AddressSanitizer and LeakSanitizer. */
#ifndef ORC_ALLOC_HOOK_H
#define ORC_ALLOC_HOOK_H
#include <stddef.h>
#include <stdlib.h>
void *orc_hook_malloc(size_t n);
void *orc_hook_calloc(size_t n, size_t size);
#define malloc(n) orc_hook_malloc(n)
#define calloc(n, size) orc_hook_calloc(n, size)
#endif
