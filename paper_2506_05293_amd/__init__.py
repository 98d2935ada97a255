"""MI355X-native D2Q9 lattice Boltzmann step with Zou & He and neural
outflow boundaries (Bedrunka et al., arXiv 2506.05293).

The compute path lives in the C-ABI library ``liblbm.so`` (HIP for gfx950);
``paper_2506_05293_amd.lbm`` is its thin ctypes binding.  Importing this
package loads nothing: the library is loaded on first use, and every entry
point raises if it is missing.
"""
