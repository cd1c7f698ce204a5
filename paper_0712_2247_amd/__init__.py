"""MI355X-native hard-sphere lattice Boltzmann step (D3Q19 BGK collide-and-stream
with the Enskog-like nonlocal hard-sphere force), served by the HIP library
``libhslb.so`` through its C ABI."""
