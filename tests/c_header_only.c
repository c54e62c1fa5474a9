/* The public header on its own, as strict C99 (no HIP headers needed). */
#include "fhesnn.h"

int main(void) { return FS_OK; }
