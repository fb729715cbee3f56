// Tile-kernel variants for int64 entries (see wht_tile.hpp).
// Name: C<TB> = contiguous pass over tiles of 2^TB entries; S<TB>c<CB> =
// strided pass over tiles of 2^(TB-CB) rows x 2^CB contiguous columns, so it
// transforms up to TB-CB index bits per pass.
#include "fwht_internal.hpp"
#include "wht_contig16.hpp"
#include "wht_tile.hpp"

namespace fwht {

std::vector<Variant> variants_u64()
{
    using S = uint64_t;
    return {
        Variant{"C11", 11, 5, 128, true, &launch_tile<11, 5, 128, true, S, false>},
        Variant{"C12", 12, 5, 256, true, &launch_tile<12, 5, 256, true, S, false>},
        Variant{"C13", 13, 5, 512, true, &launch_tile<13, 5, 512, true, S, false>},
        Variant{"C14", 14, 5, 512, true, &launch_tile<14, 5, 512, true, S, false>},
        // 2^15-entry (256 KiB) strided tiles held in registers with two-round
        // transposes (wht_contig16.hpp), full height only
        Variant{"S15c6", 15, 6, 1024, false, &launch_pinned16<S, 6, 0>, true},
        Variant{"S15c7", 15, 7, 1024, false, &launch_pinned16<S, 7, 0>, true},
        Variant{"S15c6n", 15, 6, 1024, false, &launch_pinned16<S, 6, NT_LOAD | NT_STORE>, true},
        Variant{"S15c7n", 15, 7, 1024, false, &launch_pinned16<S, 7, NT_LOAD | NT_STORE>, true},
        // 2^14-entry tiles in 512 threads, two workgroups per CU
        Variant{"C14p", 14, 5, 512, true, &launch_contig15p<S>, true},
        Variant{"C14pn", 14, 5, 512, true, &launch_contig15p<S, NT_LOAD | NT_STORE>, true},
        Variant{"S14c6p", 14, 6, 512, false, &launch_strided14p<S, 6>, true},
        Variant{"S14c6pn", 14, 6, 512, false, &launch_strided14p<S, 6, NT_LOAD | NT_STORE>, true},
        Variant{"S7c4", 7, 4, 64, false, &launch_tile<7, 4, 64, false, S, false>},
        Variant{"S8c4", 8, 4, 64, false, &launch_tile<8, 4, 64, false, S, false>},
        Variant{"S9c4", 9, 4, 64, false, &launch_tile<9, 4, 64, false, S, false>},
        Variant{"S10c4", 10, 4, 64, false, &launch_tile<10, 4, 64, false, S, false>},
        Variant{"S11c4", 11, 4, 128, false, &launch_tile<11, 4, 128, false, S, false>},
        Variant{"S12c4", 12, 4, 256, false, &launch_tile<12, 4, 256, false, S, false>},
        Variant{"S13c4", 13, 4, 512, false, &launch_tile<13, 4, 512, false, S, false>},
        Variant{"S7c5", 7, 5, 64, false, &launch_tile<7, 5, 64, false, S, false>},
        Variant{"S8c5", 8, 5, 64, false, &launch_tile<8, 5, 64, false, S, false>},
        Variant{"S9c5", 9, 5, 64, false, &launch_tile<9, 5, 64, false, S, false>},
        Variant{"S10c5", 10, 5, 64, false, &launch_tile<10, 5, 64, false, S, false>},
        Variant{"S11c5", 11, 5, 128, false, &launch_tile<11, 5, 128, false, S, false>},
        Variant{"S12c5", 12, 5, 256, false, &launch_tile<12, 5, 256, false, S, false>},
        Variant{"S13c5", 13, 5, 512, false, &launch_tile<13, 5, 512, false, S, false>},
        Variant{"S14c5", 14, 5, 512, false, &launch_tile<14, 5, 512, false, S, false>},
        Variant{"S7c6", 7, 6, 64, false, &launch_tile<7, 6, 64, false, S, false>},
        Variant{"S8c6", 8, 6, 64, false, &launch_tile<8, 6, 64, false, S, false>},
        Variant{"S9c6", 9, 6, 64, false, &launch_tile<9, 6, 64, false, S, false>},
        Variant{"S10c6", 10, 6, 64, false, &launch_tile<10, 6, 64, false, S, false>},
        Variant{"S11c6", 11, 6, 128, false, &launch_tile<11, 6, 128, false, S, false>},
        Variant{"S12c6", 12, 6, 256, false, &launch_tile<12, 6, 256, false, S, false>},
        Variant{"S13c6", 13, 6, 512, false, &launch_tile<13, 6, 512, false, S, false>},
        Variant{"S14c6", 14, 6, 512, false, &launch_tile<14, 6, 512, false, S, false>},
        Variant{"S8c7", 8, 7, 64, false, &launch_tile<8, 7, 64, false, S, false>},
        Variant{"S9c7", 9, 7, 64, false, &launch_tile<9, 7, 64, false, S, false>},
        Variant{"S10c7", 10, 7, 64, false, &launch_tile<10, 7, 64, false, S, false>},
        Variant{"S11c7", 11, 7, 128, false, &launch_tile<11, 7, 128, false, S, false>},
        Variant{"S12c7", 12, 7, 256, false, &launch_tile<12, 7, 256, false, S, false>},
        Variant{"S13c7", 13, 7, 512, false, &launch_tile<13, 7, 512, false, S, false>},
        Variant{"S14c7", 14, 7, 512, false, &launch_tile<14, 7, 512, false, S, false>},
        // the 2^14-entry tiles held by 1024 threads (16 entries each, twice the waves per CU)
        Variant{"S14c5w", 14, 5, 1024, false, &launch_tile<14, 5, 1024, false, S, false>},
        Variant{"S14c6w", 14, 6, 1024, false, &launch_tile<14, 6, 1024, false, S, false>},
        Variant{"S14c7w", 14, 7, 1024, false, &launch_tile<14, 7, 1024, false, S, false>},
        // twins with non-temporal loads and stores (the autotuner picks per size)
        Variant{"S12c4n", 12, 4, 256, false, &launch_tile<12, 4, 256, false, S, NT_LOAD | NT_STORE>},
        Variant{"S13c4n", 13, 4, 512, false, &launch_tile<13, 4, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S12c5n", 12, 5, 256, false, &launch_tile<12, 5, 256, false, S, NT_LOAD | NT_STORE>},
        Variant{"S13c5n", 13, 5, 512, false, &launch_tile<13, 5, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c5n", 14, 5, 512, false, &launch_tile<14, 5, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S12c6n", 12, 6, 256, false, &launch_tile<12, 6, 256, false, S, NT_LOAD | NT_STORE>},
        Variant{"S13c6n", 13, 6, 512, false, &launch_tile<13, 6, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c6n", 14, 6, 512, false, &launch_tile<14, 6, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S12c7n", 12, 7, 256, false, &launch_tile<12, 7, 256, false, S, NT_LOAD | NT_STORE>},
        Variant{"S13c7n", 13, 7, 512, false, &launch_tile<13, 7, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c7n", 14, 7, 512, false, &launch_tile<14, 7, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c5wn", 14, 5, 1024, false, &launch_tile<14, 5, 1024, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c6wn", 14, 6, 1024, false, &launch_tile<14, 6, 1024, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c7wn", 14, 7, 1024, false, &launch_tile<14, 7, 1024, false, S, NT_LOAD | NT_STORE>},
    };
}

}  // namespace fwht
