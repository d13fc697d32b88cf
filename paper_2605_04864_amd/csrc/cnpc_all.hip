// Single translation unit of the library: device symbols (the twiddle table)
// are shared by every kernel without relocatable device code.
#include "fft.hip"
#include "paint.hip"
#include "spectra.hip"
#include "bispec.hip"
#include "api.hip"
#include "batch.hip"
#include "sugiyama.hip"
