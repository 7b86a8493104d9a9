"""CPU FP64 oracle for the Multi-reference Cosine (MRC) method.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import, call, link or execute anything in this
package. The product path (the HIP library and its Python binding) never
touches it, and this package imports nothing from the product.

Modules
  mrc          term counts, document frequency, idf, the frequency-sorted term
               list, reference selection and partitioning, MRC signatures,
               signature normalisation, all-pairs MRC comparison, query top-K,
               BF16/FP8 quantisation and the FP32 rescoring chain
  comparators  exact TF-IDF cosine (the ground truth), Simhash-64 and Hamming
               distance, MAE/variance and recall/precision
  brute        pure-Python loops for tiny corpora, used to check `mrc`
  trigram      character 3-gram ids of raw text (the front end before counting)
  fma_chain.c  the FP32 multiply-add chain that defines the plain FP32 score

Every function names the passage of the paper it follows. Where the paper is
silent or garbled, the reading taken is stated in the docstring.

Pins (what the tests check this package against, beyond itself): brute-force
loops on tiny corpora; scikit-learn's smoothed TF-IDF transformer and cosine
(library routines for the textbook definitions); the reduction of MRC to exact
cosine when every selected term is its own reference part; closed forms for
k = 1; self-similarity, symmetry, range and bag-of-words invariances;
torch's bfloat16 / float8_e4m3fn conversions for the quantisers; exact
rational arithmetic for the FP32 multiply-add chain; hashlib's MD5 and the
stated tie rule for Simhash.
"""
